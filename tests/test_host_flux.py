"""The HIP library's face flux (paper_1302_2132_amd/csrc/gks_flux.hpp: reconstruction-free,
one face in the face-local frame) built for the host with plain arithmetic
(tests/host_flux.cpp) against the oracle's face flux, on seeded random faces: 2D and 3D,
the FP64 and FP32-flux forms, both time-weight modes (eps = tau/dt and the tau_hat mode) and
the multi-dimensional expansion, with and without the artificial relaxation time C_a.  The
faces carry steep one-sided slopes, and dt/tau spans 1e-6 to 10, so both branches of the
Kogan weights (series and exponential) are taken.  On the CPU this ties the library's
closed-form flux (closed-form moments and moment-system solutions) to the oracle's
generic evaluation (monomial moments, elimination) without a GPU; the GPU tests compare
the whole step on the device.

Bounds, per component, against p dt (the size of the flux; p about 1 here): FP64 1e-13
(measured 2e-14: rounding order only); FP32 flux 5e-5 (measured 8e-6: FP32 rounding of the
non-equilibrium terms, which these steep faces make a sizeable share of the flux)."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DP = C.POINTER(C.c_double)


@pytest.fixture(scope="module")
def hf(tmp_path_factory):
    lib = str(tmp_path_factory.mktemp("hf") / "libhost_flux.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math",
                           "-I", os.path.join(ROOT, "paper_1302_2132_amd", "csrc"), "-o", lib,
                           os.path.join(ROOT, "tests", "host_flux.cpp")])
    L = C.CDLL(lib)
    for f in (L.hf_face_flux, L.hf_face_flux_source):
        f.argtypes = [C.c_int, C.c_int, C.c_int] + [DP] * 11
        f.restype = C.c_int
    return L


def _p(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(DP)


def _cons(rho, U, p, g=1.4):
    U = np.asarray(U, dtype=np.float64)
    return np.array([rho, *(rho * U), p / (g - 1) + 0.5 * rho * float(U @ U)])


def _face(dim, rng, multid):
    nv = dim + 2
    h = 10 ** rng.uniform(-3, -1.5)
    cells = [_cons(1 + 0.2 * rng.uniform(-1, 1), 0.8 * rng.uniform(-1, 1, dim), 1 + 0.2 * rng.uniform(-1, 1))
             for _ in range(4)]
    d = [(cells[o + 1] - cells[o]) / h for o in range(3)]
    mm = lambda a, b: np.where(a * b > 0, np.sign(a) * np.minimum(abs(a), abs(b)), 0.0)  # noqa: E731
    sl, sr = mm(d[0], d[1]), mm(d[1], d[2])
    f = dict(Wl=cells[1] + sl * h / 2, Wr=cells[2] - sr * h / 2, sl=sl, sr=sr, Wi=cells[1], Wi1=cells[2],
             tl=None, tr=None, dx=h / 2, mu=10 ** rng.uniform(-5, -2), dt=10 ** rng.uniform(-4.5, -2.5) * h,
             kf=10 ** rng.uniform(-6, -2), wf=10 ** rng.uniform(0, 2), Sf=10 ** rng.uniform(-1, 2),
             c_a=float(rng.choice([0.0, 0.5])))
    if multid:
        f["tl"], f["tr"] = np.zeros((2, 5)), np.zeros((2, 5))
        f["tl"][:dim - 1, :nv] = 0.05 * rng.uniform(-1, 1, (dim - 1, nv)) * cells[1] / h
        f["tr"][:dim - 1, :nv] = 0.05 * rng.uniform(-1, 1, (dim - 1, nv)) * cells[2] / h
    return f


@pytest.mark.parametrize("mode", [0, 1, 4, 5], ids=["dt", "tauhat", "multid", "multid-tauhat"])
@pytest.mark.parametrize("fp32", [0, 1], ids=["fp64", "fp32_flux"])
@pytest.mark.parametrize("dim", [2, 3])
def test_library_flux_matches_the_oracle(hf, dim, fp32, mode):
    rng = np.random.default_rng(100 * dim + 10 * fp32 + mode)
    nv = dim + 2
    tol = 5e-5 if fp32 else 1e-13
    worst = 0.0
    for _ in range(200):
        f = _face(dim, rng, mode & 4)
        F = np.zeros(nv)
        gp = np.array([1.4, 0.72, f["mu"], f["c_a"], 0.09])
        sc = np.array([f["dx"], f["dx"], f["kf"], f["wf"], f["Sf"], f["dt"]])
        st = hf.hf_face_flux(dim, fp32, mode, _p(gp), *[_p(f[k]) for k in ("Wl", "Wr", "sl", "sr", "Wi", "Wi1")],
                             _p(f["tl"]), _p(f["tr"]), _p(sc), F.ctypes.data_as(DP))
        assert st == 0
        md = bool(mode & 4)
        ref = oracle.face_flux(dim, f["Wl"], f["Wr"], f["sl"], f["sr"], f["Wi"], f["Wi1"], f["dx"], f["dx"],
                               f["kf"], f["wf"], f["Sf"], f["dt"], mu=f["mu"], c_a=f["c_a"],
                               eps_mode="tauhat" if mode & 1 else "dt",
                               tsl=f["tl"][:dim - 1, :nv] if md else None,
                               tsr=f["tr"][:dim - 1, :nv] if md else None)["F"]
        pmax = max(0.4 * (w[-1] - 0.5 * float(w[1:nv - 1] @ w[1:nv - 1]) / w[0]) for w in (f["Wl"], f["Wr"]))
        worst = max(worst, float(np.max(np.abs(F - ref))) / (pmax * f["dt"]))
    assert worst <= tol, worst


def test_non_physical_state_is_reported_by_both(hf):
    """A face state with negative pressure: the library's flux returns 1, the oracle refuses."""
    w = _cons(1.0, [0.3, 0.0], 1.0)
    bad = w.copy()
    bad[-1] = 0.01                                # kinetic energy above the total energy
    z = np.zeros(4)
    F = np.zeros(4)
    gp = np.array([1.4, 0.72, 1e-3, 0.0, 0.09])
    sc = np.array([0.01, 0.01, 1e-3, 10.0, 1.0, 1e-4])
    assert hf.hf_face_flux(2, 0, 0, _p(gp), _p(bad), _p(w), _p(z), _p(z), _p(w), _p(w), None, None, _p(sc),
                           F.ctypes.data_as(DP)) == 1
    with pytest.raises(oracle.OracleError):
        oracle.face_flux(2, bad, w, z, z, w, w, 0.01, 0.01, 1e-3, 10.0, 1.0, 1e-4)


@pytest.mark.parametrize("mode", [0, 1, 4, 5], ids=["dt", "tauhat", "multid", "multid-tauhat"])
@pytest.mark.parametrize("fp32", [0, 1], ids=["fp64", "fp32_flux"])
@pytest.mark.parametrize("dim", [2, 3])
def test_cell_states_through_the_optional_source(hf, dim, fp32, mode):
    """The 2D tile kernel hands the flux the two cells' states through an optional source
    (read again from LDS where they are used) rather than the FaceIn copies.  With the
    copies spoiled (NaN), the flux through the source must equal the default one bitwise:
    every use of the cells' states goes through the source, and nothing else changes."""
    rng = np.random.default_rng(700 + 100 * dim + 10 * fp32 + mode)
    nv = dim + 2
    for _ in range(100):
        f = _face(dim, rng, mode & 4)
        gp = np.array([1.4, 0.72, f["mu"], f["c_a"], 0.09])
        sc = np.array([f["dx"], f["dx"], f["kf"], f["wf"], f["Sf"], f["dt"]])
        args = [_p(gp)] + [_p(f[k]) for k in ("Wl", "Wr", "sl", "sr", "Wi", "Wi1")] + [_p(f["tl"]), _p(f["tr"]),
                                                                                      _p(sc)]
        Fa, Fb = np.zeros(nv), np.zeros(nv)
        sa = hf.hf_face_flux(dim, fp32, mode, *args, Fa.ctypes.data_as(DP))
        sb = hf.hf_face_flux_source(dim, fp32, mode, *args, Fb.ctypes.data_as(DP))
        assert sa == sb == 0
        assert np.array_equal(Fa, Fb), (Fa, Fb)
