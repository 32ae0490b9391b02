"""Pins of the oracle's fifth-order WENO face values (reconstruction "weno5": the paper's
fifth-order WENO among its reconstruction schemes, section on the implementation; Jiang and
Shu's weights and smoothness indicators, applied to the conservative variables in index
space, gradients still minmod) against what the definition and the mathematics fix.

* An independent construction from the definition: each candidate is the parabola with the
  three cell averages of its stencil (a 3 x 3 solve on monomials), its smoothness indicator
  the integral over the face's upwind cell of its squared first and second derivatives,
  and the linear weights the combination of the candidates that equals the quartic through
  all five averages (a least-squares solve that must be exact).  The oracle's closed forms
  must agree with it on random data.
* Exactness: any quadratic's face value is reproduced whatever the weights.
* Order: on smooth data the face-value error falls like h^5.
* Essentially non-oscillatory: beside a jump the value is the smooth side's.
* Mirror: the right value is the left value of the mirrored data; the gradients are the
  minmod ones of the other schemes.
* The third ghost layer follows the boundary rules; runs keep a free stream and conserve.
* In the whole scheme: a convected density wave converges at second order (the time
  integration's) with well under half the third-order MUSCL error; Sod converges, below the
  minmod scheme's error.
"""
import numpy as np
import pytest

import oracle
from inputs import cases as C

EPS = 1e-6     # Jiang and Shu's epsilon, a constant of the published method


def _cell_avg_rows(cells):
    """Rows M[j, n] = average of x^n over the unit cell centred at j (n = 0, 1, 2)."""
    M = np.zeros((len(cells), 3))
    for r, j in enumerate(cells):
        for n in range(3):
            M[r, n] = ((j + 0.5) ** (n + 1) - (j - 0.5) ** (n + 1)) / (n + 1)
    return M


def _weno5_from_definition(v):
    """Face value at x = 1/2 between cells 0 and 1 of cell averages v[0..4] on the unit
    cells centred at -2 .. 2."""
    v = np.asarray(v, dtype=np.float64)
    q, beta, rows = [], [], []
    for k in range(3):
        cells = [k - 2, k - 1, k]
        A = _cell_avg_rows(cells)
        Ainv = np.linalg.inv(A)
        c = Ainv @ v[k:k + 3]                    # p(x) = c0 + c1 x + c2 x^2
        q.append(c[0] + c[1] * 0.5 + c[2] * 0.25)
        # the candidate's face value as a linear form of all five averages
        row = np.zeros(5)
        row[k:k + 3] = np.array([1.0, 0.5, 0.25]) @ Ainv
        rows.append(row)
        # smoothness: int over [-1/2, 1/2] of p'^2 + p''^2 (unit width)
        p1 = np.polynomial.Polynomial([c[1], 2.0 * c[2]])
        p2 = np.polynomial.Polynomial([2.0 * c[2]])
        b = 0.0
        for d in (p1, p2):
            I = (d * d).integ()
            b += I(0.5) - I(-0.5)
        beta.append(b)
    # linear weights: the candidates' combination equal to the quartic through all five
    M5 = np.zeros((5, 5))
    for r, j in enumerate(range(-2, 3)):
        for n in range(5):
            M5[r, n] = ((j + 0.5) ** (n + 1) - (j - 0.5) ** (n + 1)) / (n + 1)
    quartic_row = np.array([0.5 ** n for n in range(5)]) @ np.linalg.inv(M5)
    d, *_ = np.linalg.lstsq(np.array(rows).T, quartic_row, rcond=None)
    assert np.allclose(np.array(rows).T @ d, quartic_row, atol=1e-13)
    alpha = d / (EPS + np.array(beta)) ** 2
    return float(alpha @ np.array(q) / alpha.sum()), d


def test_linear_weights_of_the_definition():
    _, d = _weno5_from_definition(np.arange(5.0))
    assert np.allclose(d, [0.1, 0.6, 0.3], atol=1e-13)


@pytest.mark.parametrize("scale", [1.0, 1e-3, 50.0])
def test_closed_forms_match_the_definition(scale):
    rng = np.random.default_rng(int(scale * 1000) + 7)
    for _ in range(40):
        v = scale * rng.uniform(-1.0, 1.0, size=5)
        want, _ = _weno5_from_definition(v)
        got = oracle.weno5(v)
        assert abs(got - want) <= 1e-12 * max(np.max(np.abs(v)), 1e-300), (v, got, want)


def test_epsilon_matters_for_nearly_linear_data():
    """Smoothness indicators near epsilon: the value depends on epsilon itself."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        v = 0.2 * np.arange(5.0) + 3e-4 * rng.uniform(-1, 1, size=5)
        want, _ = _weno5_from_definition(v)
        assert abs(oracle.weno5(v) - want) <= 1e-13


@pytest.mark.parametrize("seed", range(4))
def test_quadratics_are_exact(seed):
    rng = np.random.default_rng(seed)
    A, B, Cc = rng.uniform(-2, 2, size=3)
    h = rng.uniform(0.1, 3.0)
    j = np.arange(-2, 3)
    v = A + B * h * j + Cc * h * h * (j * j + 1.0 / 12.0)      # averages of A + B x + C x^2 over cells of width h
    exact = A + B * h * 0.5 + Cc * h * h * 0.25
    assert abs(oracle.weno5(v) - exact) <= 1e-13 * (abs(A) + abs(B * h) + abs(Cc * h * h))


def test_fifth_order_on_smooth_data():
    F = lambda x: -np.cos(x) + 0.15 * x * x             # noqa: E731  antiderivative of sin x + 0.3 x
    f = lambda x: np.sin(x) + 0.3 * x                    # noqa: E731
    x0, errs = 0.3, []
    hs = [0.2, 0.1, 0.05, 0.025]
    for h in hs:
        j = np.arange(-2, 3)
        v = (F(x0 + (j + 0.5) * h) - F(x0 + (j - 0.5) * h)) / h
        errs.append(abs(oracle.weno5(v) - f(x0 + 0.5 * h)))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders[1:]) > 4.6, (errs, orders)


@pytest.mark.parametrize("jump", [9.0, -0.7])
def test_value_beside_a_jump_is_the_smooth_sides(jump):
    """Upwind cells constant, a jump across the face: the face value is that constant."""
    v = np.array([1.0, 1.0, 1.0, 1.0 + jump, 1.0 + jump])
    assert abs(oracle.weno5(v) - 1.0) <= 1e-9
    # linear data with a jump one cell further downwind: only the candidate that crosses it
    # is wrong, and its weight falls with the square of its smoothness indicator
    v = np.array([2.0, 2.5, 3.0, 3.5, 3.5 + 10 * jump])
    assert abs(oracle.weno5(v) - 3.25) <= 1e-5 * abs(10 * jump)


def test_mirror_and_minmod_gradients():
    rng = np.random.default_rng(11)
    for _ in range(10):
        w = rng.uniform(0.5, 2.0, size=6)
        xc = np.cumsum(rng.uniform(0.5, 1.5, size=4))
        xf = 0.5 * (xc[1] + xc[2])
        wl, wr, sl, sr = oracle.reconstruct("weno5", w, xc, xf)
        assert wl == oracle.weno5(w[0:5])
        assert wr == oracle.weno5(w[5:0:-1])
        # mirrored data: the roles of the two sides swap
        wl2, wr2, sl2, sr2 = oracle.reconstruct("weno5", w[::-1], (xc[-1] + xc[0]) - xc[::-1], (xc[-1] + xc[0]) - xf)
        assert wl2 == wr and wr2 == wl
        # the gradients are those of the second-order scheme on the inner four cells
        g = oracle.reconstruct("muscl2", w[1:5], xc, xf)
        assert (sl, sr) == (g[2], g[3])


def test_third_ghost_layer_follows_the_boundary_rules():
    n = (7, 5, 1)
    bc = [["wall", "outflow"], ["periodic", "periodic"]]
    c = C.uniform_flow(dim=2, n=n, bc=bc, seed=4)
    rng = np.random.default_rng(2)
    c.W = c.W * (1.0 + 0.1 * rng.uniform(-1, 1, size=c.W.shape))
    c.recon = "weno5"
    We = oracle.ghost_fill(c)                        # (nv, 1, ny + 6, nx + 6)
    W = c.W[:, 0]
    E = We[:, 0]
    g = 3
    # x low wall: cell -1-i mirrors cell i, momentum negated; x high outflow copies
    for i in range(3):
        mir = W[:, :, i].copy()
        mir[1:3] *= -1.0
        assert np.array_equal(E[:, g:g + n[1], g - 1 - i], mir)
        assert np.array_equal(E[:, g:g + n[1], g + n[0] + i], W[:, :, n[0] - 1])
    # y periodic: row -3 is row n-3, row n+2 is row 2
    assert np.array_equal(E[:, g - 3, g:g + n[0]], W[:, n[1] - 3, :])
    assert np.array_equal(E[:, g + n[1] + 2, g:g + n[0]], W[:, 2, :])


def _entropy_errors(recon):
    errs = []
    for N in (32, 64, 128):
        case = C.entropy_wave(N, t_end=0.5, ny=3)
        case.recon = recon
        r = oracle.run(case, 10 ** 6, nthreads=8)
        assert r["t"] == 0.5
        xf = case.xf[0]
        dx = np.diff(xf)
        xa, xb = xf[:-1] - 0.5, xf[1:] - 0.5
        exact = 1.0 - 0.2 * (np.cos(2 * np.pi * xb) - np.cos(2 * np.pi * xa)) / (2 * np.pi * dx)
        errs.append(float(np.mean(np.abs(r["W"][0, 0, 0] - exact))))
    return errs


def test_entropy_wave_with_weno5_face_values():
    """A convected density wave (exact: the initial cell averages shifted): second order
    overall (the time integration is second order), with well under half the error of the
    third-order MUSCL face values at every resolution."""
    e5, e3 = _entropy_errors("weno5"), _entropy_errors("muscl3")
    assert np.log2(e5[1] / e5[2]) > 1.9, e5
    assert all(a < 0.5 * b for a, b in zip(e5, e3)), (e5, e3)


def test_sod_converges_with_weno5():
    import exact_riemann as ER
    errs, errs2 = [], []
    for N in (100, 200):
        for recon, out in (("weno5", errs), ("muscl2", errs2)):
            case = C.sod_tube(N, ny=3, t_end=0.2)
            case.recon = recon
            r = oracle.run(case, 100000, nthreads=8)
            x = 0.5 * (case.xf[0][1:] + case.xf[0][:-1])
            ex = ER.sample((1, 0, 1), (0.125, 0, 0.1), x, 0.2)
            out.append(float(np.mean(np.abs(r["W"][0, 0, 0] - ex[0]))))
    assert errs[1] < 0.65 * errs[0] < 0.02, errs
    assert all(a < b for a, b in zip(errs, errs2)), (errs, errs2)


def test_free_stream_and_conservation():
    bc = [["dirichlet", "outflow"], ["outflow", "profile"]]
    c = C.uniform_flow(dim=2, n=(12, 9, 1), bc=bc, seed=8)
    c.recon = "weno5"
    r = oracle.run(c, 4)
    assert np.max(np.abs(r["W"] - c.W)) <= 1e-14 * np.max(np.abs(c.W))
    m = C.mixing_layer(24, seed=7)
    m.recon = "weno5"
    vol = np.outer(np.diff(m.xf[1]), np.diff(m.xf[0]))
    r = oracle.run(m, 8)
    for k in range(4):
        before, after = np.sum(m.W[k, 0] * vol), np.sum(r["W"][k, 0] * vol)
        assert abs(after - before) <= 1e-13 * np.sum(np.abs(m.W[k, 0]) * vol)
    m2 = m.copy()
    m2.recon = "muscl2"
    assert np.max(np.abs(oracle.run(m2, 8)["W"] - r["W"])) > 1e-8


def test_fewer_than_three_cells_refused():
    c = C.uniform_flow(dim=2, n=(2, 5, 1), bc=[["periodic", "periodic"]] * 2)
    c.recon = "weno5"
    with pytest.raises(oracle.OracleError):
        oracle.run(c, 1)

