"""Helpers shared by the GPU tests: run a case through libgks and compare with the oracle."""
import numpy as np


def field_errors(got, ref, vector_momentum=False):
    """Per-field normwise relative error max_i |got - ref| / max_i |ref|.

    With vector_momentum, each momentum component is scaled by the largest momentum
    magnitude |rho U| instead of its own largest value (a rotation-invariant scale: a
    component that is a small perturbation is not measured against itself)."""
    nv = ref.shape[0]
    dim = nv - 2
    mom = np.sqrt(sum(ref[1 + d] ** 2 for d in range(dim)))
    out = []
    for m in range(nv):
        if vector_momentum and 1 <= m <= dim:
            scale = float(np.max(mom))
        else:
            scale = float(np.max(np.abs(ref[m])))
        scale = max(scale, 1e-300)
        out.append(float(np.max(np.abs(got[m] - ref[m]))) / scale)
    return np.array(out)


def run_gpu(case, nsteps, which="cons"):
    from paper_1302_2132_amd import Solver
    s = Solver(case)
    try:
        s.step(nsteps)
        r = s.residual()
        W = s.fields(which)
    finally:
        s.close()
    return W, r


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
