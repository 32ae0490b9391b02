"""The operation-counting build of the oracle (oracle/opcount.cpp: the oracle's source with
its scalar type replaced by a counting one) computes the oracle's fluxes bitwise and counts
each kind of operation of one face flux.  The counts are the oracle's own, independent of
the HIP library's count of its closed-form evaluation (gks_face_flops): the oracle builds
its moments from generic monomial tables and solves each moment system by elimination, so
it takes several times the kernel's operations; the roofline uses the smaller count."""
import numpy as np
import pytest

import oracle


def _face(dim, seed=0):
    rng = np.random.default_rng(seed)
    nv = dim + 2

    def cons(rho, U, p, g=1.4):
        return np.array([rho, *(rho * np.asarray(U)), p / (g - 1) + 0.5 * rho * float(np.dot(U, U))])

    cells = [cons(1.0 + 0.1 * rng.uniform(-1, 1), 0.3 * rng.uniform(-1, 1, dim), 0.9 + 0.1 * rng.uniform(-1, 1))
             for _ in range(4)]
    h = 0.01
    d = [(cells[o + 1] - cells[o]) / h for o in range(3)]
    mm = lambda a, b: np.where(a * b > 0, np.sign(a) * np.minimum(abs(a), abs(b)), 0.0)  # noqa: E731
    sl, sr = mm(d[0], d[1]), mm(d[1], d[2])
    args = (dim, cells[1] + sl * h / 2, cells[2] - sr * h / 2, sl, sr, cells[1], cells[2], h / 2, h / 2,
            1e-3, 10.0, 5.0, 3e-3)
    assert all(len(a) == nv for a in args[1:7])
    return args


@pytest.mark.parametrize("dim,mode", [(2, "dt"), (3, "dt"), (2, "tauhat"), (3, "tauhat")])
def test_counting_build_computes_the_oracle_bitwise(dim, mode):
    args = _face(dim, seed=dim)
    counts, F = oracle.face_op_counts(*args, mu=1e-3, c_a=0.1, eps_mode=mode)
    ref = oracle.face_flux(*args, mu=1e-3, c_a=0.1, eps_mode=mode)["F"]
    assert np.array_equal(F, ref)
    assert set(counts) == set(oracle.OP_KINDS)


def test_operation_counts_of_a_face():
    from paper_1302_2132_amd import gks_face_flops
    for dim in (2, 3):
        counts, _ = oracle.face_op_counts(*_face(dim), mu=1e-3, c_a=0.1)
        total = sum(counts.values())
        print(dim, counts, total)
        # three half-line or full-line moment sets need an erfc each (left, right, interface,
        # and the equilibrium's two halves), the Maxwellians' exponentials and the time weights
        assert counts["erfc"] >= 3 and counts["exp"] >= 3 and counts["sqrt"] >= 2
        # the oracle's generic evaluation takes more operations than the kernel's closed form
        assert total > 2 * gks_face_flops(dim)
    c2, _ = oracle.face_op_counts(*_face(2), mu=1e-3, c_a=0.1)
    c3, _ = oracle.face_op_counts(*_face(3), mu=1e-3, c_a=0.1)
    assert sum(c3.values()) > sum(c2.values())
