"""Helpers shared by the GPU tests: run a case through libgks and compare with the oracle."""
import numpy as np


def field_errors(got, ref):
    """Per-field normwise relative error max_i |got - ref| / max_i |ref|."""
    nv = ref.shape[0]
    out = []
    for m in range(nv):
        scale = max(float(np.max(np.abs(ref[m]))), 1e-300)
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
