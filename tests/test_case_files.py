"""Case files (Case.save / Case.load: JSON for sizes, boundary names, gas and run
parameters and options, .npz for the arrays): every generator's case comes back bitwise,
gives the same C-ABI configuration (workspace size), and the oracle steps it to the same
state."""
import dataclasses

import numpy as np
import pytest

import oracle
from inputs import cases as C


def _cases():
    ml = C.mixing_layer(16, seed=2)
    sb = C.sbli(24, 12, precision="fp32_flux")
    sb.kw_transport, sb.recon = True, "muscl3"
    bx = C.isotropic_box(6, precision="fp64")
    bx.eps_mode, bx.recon = "tauhat", "weno5"
    st = C.shock_tube(20, 4, shift=0.8, t_end=0.05)
    bc = [["dirichlet", "outflow"], ["wall", "profile"], ["outflow", "wall"]]
    uf = C.uniform_flow(dim=3, n=(5, 4, 3), bc=bc, vel=(0.4, 0.1, -0.2))
    uf.multi_d, uf.res_tol, uf.max_steps = True, 1e-6, 7
    return [ml, sb, bx, st, uf] + C.batch_cases(3, seed=5, nmin=16, nmax=24)


@pytest.mark.parametrize("i", range(8))
def test_case_round_trip(tmp_path, i):
    import paper_1302_2132_amd as P
    c = _cases()[i]
    path = str(tmp_path / "case.json")
    c.save(path)
    d = C.Case.load(path)
    for f in dataclasses.fields(C.Case):
        a, b = getattr(c, f.name), getattr(d, f.name)
        if f.name in ("W", "k", "omega"):
            assert a.dtype == b.dtype and np.array_equal(a, b), f.name
        elif f.name == "xf":
            assert all(np.array_equal(x, y) for x, y in zip(a, b))
        elif f.name == "bc_data":
            for p, q in zip(a, b):
                for x, y in zip(p, q):
                    assert (x is None) == (y is None) and (x is None or np.array_equal(x, y))
        elif f.name == "meta":
            assert b == {k: v for k, v in a.items() if isinstance(v, (bool, int, float, str))}
        else:
            assert list(a) == list(b) if f.name in ("n", "bc") else a == b, f.name
    assert P.gks_workspace_bytes(P.config_from_case(c)) == P.gks_workspace_bytes(P.config_from_case(d))


def test_loaded_case_steps_like_the_original(tmp_path):
    c = C.mixing_layer(12, seed=7)
    path = str(tmp_path / "ml.json")
    c.save(path)
    d = C.Case.load(path)
    a, b = oracle.run(c, 3), oracle.run(d, 3)
    assert np.array_equal(a["W"], b["W"]) and a["t"] == b["t"]
