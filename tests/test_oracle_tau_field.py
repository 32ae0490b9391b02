"""Pin of the oracle's relaxation-time field (og_tau_field, the gks_fields(TAU) reference).

On a uniform flow the strain rate vanishes, the two face states and the interface state are
the flow itself, and the pressure jump of the artificial part (Eq. taua) is zero, so the
relaxation time of every face is (Eqs. relaxation time and tautchenadjusted, T = p/rho)

    tau = (mu + rho k_f / omega_f) / p,   k_f, omega_f the means of the face's two cells,

a ghost cell taking the k and omega of its interior image (periodic: the wrapped cell;
otherwise the boundary cell).  The field is the largest tau over each cell's faces.  Random
k and omega on stretched grids, 2D and 3D, with C_a > 0 (which must not contribute here),
and every boundary type that keeps the flow uniform (a wall's mirrored ghost does not)."""
import numpy as np
import pytest

import oracle
from inputs import cases as C


def _image(i, n, periodic):
    if 0 <= i < n:
        return i
    if periodic:
        return i % n
    return 0 if i < 0 else n - 1


def _expected(case):
    dim = case.dim
    rho = case.W[0].reshape(-1)[0]
    mom = [case.W[1 + d].reshape(-1)[0] for d in range(dim)]
    p = (case.gamma - 1.0) * (case.W[dim + 1].reshape(-1)[0] - 0.5 * sum(m * m for m in mom) / rho)
    k, w = case.k, case.omega                   # (nz, ny, nx)
    out = np.zeros_like(k)
    shape = k.shape
    axis_of = {0: 2, 1: 1, 2: 0}               # grid axis d -> array axis
    for idx in np.ndindex(*shape):
        best = 0.0
        for d in range(dim):
            ax = axis_of[d]
            n = shape[ax]
            per = case.bc[d][0] == "periodic"
            for side in (-1, 1):
                nb = list(idx)
                nb[ax] = _image(idx[ax] + side, n, per)
                kf = 0.5 * (k[idx] + k[tuple(nb)])
                wf = 0.5 * (w[idx] + w[tuple(nb)])
                best = max(best, (case.mu + rho * kf / wf) / p)
        out[idx] = best
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_tau_field_of_a_uniform_flow(dim):
    if dim == 2:
        bc = [["dirichlet", "outflow"], ["outflow", "profile"]]
        c = C.uniform_flow(dim=2, n=(9, 7, 1), bc=bc, vel=(0.4, 0.1))
    else:
        bc = [["periodic", "periodic"], ["profile", "outflow"], ["dirichlet", "outflow"]]
        c = C.uniform_flow(dim=3, n=(6, 5, 4), bc=bc, vel=(0.4, 0.1, -0.2))
    c.c_a = 1.0
    got = oracle.tau_field(c)
    want = _expected(c)
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(want), (got, want)
    # and the rarefaction field of the same flow is zero (no density or velocity gradient)
    assert np.max(np.abs(oracle.eps_field(c))) <= 1e-14 * np.max(want)
