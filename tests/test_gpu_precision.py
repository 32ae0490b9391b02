"""FP32-flux form against the FP64 form at the full configurations and their stated step
counts (the FP64 GPU path itself matches the oracle within 1e-12, see test_gpu_parity).
Error per field: max |fp32 - fp64| / max |fp64|, momentum components against the largest
momentum magnitude."""
import numpy as np
import pytest

from gpu_util import banner, field_errors
from inputs import cases as C

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def _pair(make, steps):
    from paper_1302_2132_amd import Solver
    out = []
    for prec in ("fp64", "fp32_flux"):
        c = make(prec)
        s = Solver(c)
        s.step(steps)
        r = s.residual()
        out.append(s.fields("cons"))
        s.close()
        assert r["steps"] == steps
    return out


def test_sbli_1024x512_fp32_flux_2000_steps():
    banner("sbli 1024x512 fp64 vs fp32-flux, 2000 steps")
    W64, W32 = _pair(lambda p: C.sbli(precision=p), 2000)
    err = field_errors(W32, W64, vector_momentum=True)
    print(f"  errors {err} per-component {field_errors(W32, W64)}", flush=True)
    assert np.all(err <= TOL32), err


def test_isotropic_256_fp32_flux_500_steps():
    banner("isotropic 256^3 fp64 vs fp32-flux, 500 steps")
    W64, W32 = _pair(lambda p: C.isotropic_box(256, precision=p), 500)
    err = field_errors(W32, W64, vector_momentum=True)
    print(f"  errors {err} per-component {field_errors(W32, W64)}", flush=True)
    assert np.all(err <= TOL32), err


def test_batch_64_fp32_flux_200_steps():
    from paper_1302_2132_amd import Batch, Solver
    banner("64-mesh batch fp64 vs fp32-flux, 200 steps")
    res = {}
    for prec in ("fp64", "fp32_flux"):
        cases = C.batch_cases(64, seed=3, steps=200, precision=prec)
        solvers = [Solver(c) for c in cases]
        b = Batch(solvers, capacity=64)
        b.capture()
        b.step(200)
        st = b.status()
        assert np.all(st["steps"] == 200)
        res[prec] = [s.fields("cons") for s in solvers]
        b.close()
        for s in solvers:
            s.close()
    worst = np.zeros(4)
    for a, b64 in zip(res["fp32_flux"], res["fp64"]):
        worst = np.maximum(worst, field_errors(a, b64, vector_momentum=True))
    print(f"  worst errors over 64 meshes {worst}", flush=True)
    assert np.all(worst <= TOL32), worst
