"""The workspace-free batch (gks_batch_create_static) gives the results of the batch with a
caller workspace (gks_batch_create), through the C ABI, on two calls in a row, the second
with a smaller input; and its limits are enforced."""
import numpy as np
import pytest

from gpu_util import banner
from inputs import cases as C

pytestmark = pytest.mark.gpu


def _first():
    return [C.mixing_layer(40, seed=11), C.sbli(48, 24, precision="fp32_flux"),
            C.isotropic_box(10, precision="fp64"), C.mixing_layer(33, seed=12, precision="fp32_flux"),
            C.sod_tube(60, ny=2, t_end=0.02)]


def _second():
    # fewer members, fewer cells, a smaller capacity: the scratch keeps the first call's
    # larger table behind the new one
    return [C.mixing_layer(20, seed=5), C.isotropic_box(6, precision="fp32_flux")]


def _run(cases, nsteps, capacity, static, graph):
    from paper_1302_2132_amd import Batch, Solver
    solvers = [Solver(c) for c in cases]
    b = Batch(solvers, capacity=capacity, static=static)
    try:
        if graph:
            b.capture()
        b.step(nsteps)
        st = b.status()
        out = [(s.fields("cons"), s.residual()) for s in solvers]
    finally:
        b.close()
        for s in solvers:
            s.close()
    return out, st


@pytest.mark.parametrize("graph", [False, True])
def test_static_batch_equals_workspace_batch_twice(graph):
    for label, make, nsteps, capacity in (("first", _first, 14, 8), ("second, smaller", _second, 9, 2)):
        banner(f"static batch, {label} call, graph={graph}")
        cases = make()
        ref, st_ref = _run(cases, nsteps, capacity, static=False, graph=graph)
        got, st_got = _run(make(), nsteps, capacity, static=True, graph=graph)
        assert np.array_equal(st_got["steps"], st_ref["steps"])
        assert np.array_equal(st_got["state"], st_ref["state"])
        for i, ((Wg, rg), (Wr, rr)) in enumerate(zip(got, ref)):
            # bitwise: the same kernels walk the same table, only its address differs
            assert np.array_equal(Wg, Wr), (label, i, cases[i].name)
            assert np.array_equal(rg["res"], rr["res"]), (label, i)
            assert rg["t"] == rr["t"] and rg["steps"] == rr["steps"], (label, i)


def test_static_batch_limits():
    from paper_1302_2132_amd import (GKS_BATCH_STATIC_CAPACITY, GKS_ERR_ARG, GKS_ERR_STATE, Batch, GksError,
                                     Solver)
    s = Solver(C.mixing_layer(16, seed=1))
    try:
        with pytest.raises(GksError) as e:
            Batch([s], capacity=GKS_BATCH_STATIC_CAPACITY + 1, static=True)
        assert e.value.status == GKS_ERR_ARG
        b = Batch([s], capacity=4, static=True)
        with pytest.raises(GksError) as e:         # one workspace-free batch per device
            Batch([s], capacity=4, static=True)
        assert e.value.status == GKS_ERR_STATE
        b.step(3)
        assert int(b.status()["steps"][0]) == 3
        b.close()
        b = Batch([s], capacity=GKS_BATCH_STATIC_CAPACITY, static=True)   # released: usable again
        b.step(2)
        assert int(b.status()["steps"][0]) == 5
        b.close()
    finally:
        s.close()
