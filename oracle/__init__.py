"""FP64 CPU oracle of the turbulent gas-kinetic scheme -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps `gks_oracle.c` (plain C, OpenMP over faces and
cells) through ctypes and shares nothing with the HIP library except the seeded
input generators in `inputs/`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gks_oracle.c")
LIB = os.path.join(HERE, "libgks_oracle.so")

BC_CODE = {"periodic": 0, "wall": 1, "dirichlet": 2, "profile": 3, "outflow": 4}
ERRORS = {0: "ok", 1: "bad argument", 2: "nonphysical state"}
INFO_LEN = 51
EPS_MODE = {"dt": 0, "tauhat": 1}
RECON = {"muscl2": 0, "muscl3": 1, "weno5": 2}
NU = 12


def build(force: bool = True) -> str:
    """Compile the oracle: -O2, no fast math, no FP contraction, OpenMP."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-ffp-contract=off", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Case(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("n", C.c_long * 3),
        ("xf", C.c_void_p * 3),
        ("bc", (C.c_int * 2) * 3),
        ("bc_data", (C.c_void_p * 2) * 3),
        ("gamma", C.c_double), ("prandtl", C.c_double), ("mu", C.c_double),
        ("c_a", C.c_double), ("c_mu", C.c_double), ("cfl", C.c_double), ("t_end", C.c_double),
        ("eps_mode", C.c_int),
        ("recon", C.c_int),
        ("multi_d", C.c_int),
    ]


_lib = None


def use_library(path):
    """Point the wrapper at another build of the oracle (tests that plant mistakes in a
    copy of the source use this); None restores the default library."""
    global _lib
    _lib = None
    if path is not None:
        _bind(C.CDLL(path))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _bind(C.CDLL(LIB))
    return _lib


def _bind(L):
    global _lib
    _lib = L
    dp = C.POINTER(C.c_double)
    _lib.og_run.argtypes = [C.c_void_p, dp, dp, dp, C.c_int, C.c_int, dp, dp, dp, C.POINTER(C.c_long)]
    _lib.og_dt.argtypes = [C.c_void_p, dp, dp, dp, dp]
    _lib.og_strain_field.argtypes = [C.c_void_p, dp, dp]
    _lib.og_ghost_fill.argtypes = [C.c_void_p, dp, dp]
    _lib.og_step_cells.argtypes = [C.c_void_p, dp, dp, dp, C.c_double, C.POINTER(C.c_long),
                                   C.c_long, C.c_int, dp]
    _lib.og_face_flux.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp]
    _lib.og_moments_u.argtypes = [C.c_double, C.c_double, dp]
    _lib.og_kogan.argtypes = [C.c_double, C.c_double, dp]
    _lib.og_moment_solve.argtypes = [C.c_int, C.c_double, dp, dp, dp]
    _lib.og_tau_value.argtypes = [C.c_double] * 11
    _lib.og_tau_value.restype = C.c_double
    if hasattr(_lib, "og_recon"):
        _lib.og_recon.argtypes = [C.c_int, dp, dp, C.c_double, dp]
    if hasattr(_lib, "og_weno5_value"):
        _lib.og_weno5_value.argtypes = [dp]
        _lib.og_weno5_value.restype = C.c_double
    if hasattr(_lib, "og_kogan_e"):
        _lib.og_kogan_e.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        _lib.og_eps_field.argtypes = [C.c_void_p, dp, dp, dp, dp]
    if hasattr(_lib, "og_tau_field"):
        _lib.og_tau_field.argtypes = [C.c_void_p, dp, dp, dp, dp]
    if hasattr(_lib, "og_run_kw"):
        _lib.og_run_kw.argtypes = [C.c_void_p, dp, dp, dp, C.c_int, C.c_int, dp, dp, dp, C.POINTER(C.c_long)]
        _lib.og_kw_sources.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


class _Bound:
    """Keeps the ctypes case struct and the arrays it points to alive together."""

    def __init__(self, case):
        self.keep = []
        s = _Case()
        s.dim = case.dim
        for d in range(3):
            s.n[d] = int(case.n[d]) if d < case.dim else 1
        for d in range(case.dim):
            xf = np.ascontiguousarray(case.xf[d], dtype=np.float64)
            self.keep.append(xf)
            s.xf[d] = xf.ctypes.data
            for side in range(2):
                s.bc[d][side] = BC_CODE[case.bc[d][side]]
                bd = case.bc_data[d][side]
                if bd is not None:
                    bd = np.ascontiguousarray(bd, dtype=np.float64)
                    self.keep.append(bd)
                    s.bc_data[d][side] = bd.ctypes.data
        s.gamma, s.prandtl, s.mu = case.gamma, case.prandtl, case.mu
        s.c_a, s.c_mu, s.cfl, s.t_end = case.c_a, case.c_mu, case.cfl, case.t_end
        s.eps_mode = EPS_MODE[getattr(case, "eps_mode", "dt")]
        s.recon = RECON[getattr(case, "recon", "muscl2")]
        s.multi_d = 1 if getattr(case, "multi_d", False) else 0
        self.s = s

    @property
    def ptr(self):
        return C.addressof(self.s)


def _flat(a):
    return np.ascontiguousarray(a, dtype=np.float64).reshape(-1)


def run(case, nsteps=None, nthreads=0, W=None, t0=0.0):
    """Advance `case` (or W) by nsteps; returns dict(W, res, dt, t, steps)."""
    b = _Bound(case)
    Wf = _flat(case.W if W is None else W).copy()
    k, om = _flat(case.k), _flat(case.omega)
    res = np.zeros(case.nvar)
    dt = np.zeros(1)
    t = np.array([t0], dtype=np.float64)
    done = C.c_long(0)
    n = case.steps if nsteps is None else nsteps
    st = lib().og_run(b.ptr, _dp(Wf), _dp(k), _dp(om), int(n), int(nthreads), _dp(res), _dp(dt),
                      _dp(t), C.byref(done))
    if st:
        raise OracleError(st)
    return {"W": Wf.reshape(case.W.shape), "res": res, "dt": float(dt[0]), "t": float(t[0]),
            "steps": int(done.value)}


def run_kw(case, nsteps=None, nthreads=0, W=None, k=None, omega=None, t0=0.0):
    """Like run, with k and omega transported: returns dict(W, k, omega, res, dt, t, steps)."""
    b = _Bound(case)
    Wf = _flat(case.W if W is None else W).copy()
    kf = _flat(case.k if k is None else k).copy()
    wf = _flat(case.omega if omega is None else omega).copy()
    res = np.zeros(case.nvar)
    dt = np.zeros(1)
    t = np.array([t0], dtype=np.float64)
    done = C.c_long(0)
    n = case.steps if nsteps is None else nsteps
    st = lib().og_run_kw(b.ptr, _dp(Wf), _dp(kf), _dp(wf), int(n), int(nthreads), _dp(res), _dp(dt),
                         _dp(t), C.byref(done))
    if st:
        raise OracleError(st)
    return {"W": Wf.reshape(case.W.shape), "k": kf.reshape(case.k.shape), "omega": wf.reshape(case.k.shape),
            "res": res, "dt": float(dt[0]), "t": float(t[0]), "steps": int(done.value)}


def kw_sources(case, W=None, k=None, omega=None):
    """Explicit k-omega sources (Qk, Qw) of every cell."""
    b = _Bound(case)
    Wf = _flat(case.W if W is None else W)
    Qk, Qw = np.zeros(case.ncells), np.zeros(case.ncells)
    st = lib().og_kw_sources(b.ptr, _dp(Wf), _dp(_flat(case.k if k is None else k)),
                             _dp(_flat(case.omega if omega is None else omega)), _dp(Qk), _dp(Qw))
    if st:
        raise OracleError(st)
    return Qk.reshape(case.k.shape), Qw.reshape(case.k.shape)


def cfl_dt(case, W=None):
    b = _Bound(case)
    Wf = _flat(case.W if W is None else W)
    out = np.zeros(1)
    st = lib().og_dt(b.ptr, _dp(Wf), _dp(_flat(case.k)), _dp(_flat(case.omega)), _dp(out))
    if st:
        raise OracleError(st)
    return float(out[0])


def strain(case, W=None):
    b = _Bound(case)
    Wf = _flat(case.W if W is None else W)
    S = np.zeros(case.ncells)
    st = lib().og_strain_field(b.ptr, _dp(Wf), _dp(S))
    if st:
        raise OracleError(st)
    return S.reshape(case.k.shape)


def ghost_fill(case, W=None):
    b = _Bound(case)
    Wf = _flat(case.W if W is None else W)
    width = 3 if getattr(case, "recon", "muscl2") == "weno5" else 2
    g = [width if d < case.dim else 0 for d in range(3)]
    ext = [case.n[d] + 2 * g[d] if d < case.dim else 1 for d in range(3)]
    We = np.zeros(case.nvar * ext[0] * ext[1] * ext[2])
    st = lib().og_ghost_fill(b.ptr, _dp(Wf), _dp(We))
    if st:
        raise OracleError(st)
    return We.reshape(case.nvar, ext[2], ext[1], ext[0])


def step_cells(case, W, dt, cells, nthreads=0):
    """New values of the listed (flat) cells after one step of size dt from W."""
    b = _Bound(case)
    Wf = _flat(W)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), case.nvar))
    st = lib().og_step_cells(b.ptr, _dp(Wf), _dp(_flat(case.k)), _dp(_flat(case.omega)), float(dt),
                             cells.ctypes.data_as(C.POINTER(C.c_long)), len(cells), int(nthreads),
                             _dp(out))
    if st:
        raise OracleError(st)
    return out


def face_flux(dim, Wl, Wr, sl, sr, Wi, Wi1, dxl, dxr, kf, wf, Sf, dt,
              gamma=1.4, prandtl=0.72, mu=1e-3, c_a=0.0, c_mu=0.09, eps_mode="dt", tsl=None, tsr=None):
    """One interface in the face-local frame (normal velocity first).  tsl, tsr: tangential
    gradients of the two cells, (dim - 1, nv), for the multi-dimensional expansion.

    Returns dict(F, G, q, info) with info holding W0, a_l, a_r, A_l, A_r, abar_l, abar_r,
    Abar (5 slots each), tau, gam0..5, c1, c4, c5 and eps_hat (= tau/tau_hat)."""
    nv = dim + 2
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (Wl, Wr, sl, sr)]
    if tsl is not None:
        tan = []
        for t in (tsl, tsr):
            a = np.zeros((2, 5))
            a[:dim - 1, :nv] = np.asarray(t, dtype=np.float64).reshape(dim - 1, nv)
            tan.append(a)
        targs = [_dp(a) for a in tan]
    else:
        tan, targs = [], [None, None]
    wis = [np.ascontiguousarray(x, dtype=np.float64) for x in (Wi, Wi1)]
    params = np.array([gamma, prandtl, mu, c_a, c_mu, EPS_MODE[eps_mode]], dtype=np.float64)
    F, G, q, info = np.zeros(nv), np.zeros(nv), np.zeros(1), np.zeros(INFO_LEN)
    st = lib().og_face_flux(dim, _dp(params), *[_dp(a) for a in arrs], *targs, *[_dp(a) for a in wis],
                            float(dxl), float(dxr), float(kf), float(wf), float(Sf), float(dt),
                            _dp(F), _dp(G), _dp(q), _dp(info))
    if st:
        raise OracleError(st)
    names = ["W0", "a_l", "a_r", "A_l", "A_r", "abar_l", "abar_r", "Abar"]
    d = {nm: info[5 * i:5 * i + nv].copy() for i, nm in enumerate(names)}
    d.update(tau=info[40], gam=info[41:47].copy(), c=info[47:50].copy(), eps_hat=info[50])
    return {"F": F, "G": G, "q": float(q[0]), "info": d}


OPCOUNT_SRC = os.path.join(HERE, "opcount.cpp")
OPCOUNT_LIB = os.path.join(HERE, "libgks_oracle_opcount.so")
OP_KINDS = ("add", "mul", "div", "sqrt", "exp", "erfc")
_oplib = None


def build_opcount(force: bool = True) -> str:
    """Compile the operation-counting build of the oracle (opcount.cpp: the oracle's source
    with its scalar type replaced by a counting one)."""
    if force or not os.path.exists(OPCOUNT_LIB):
        cmd = ["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
               "-I", HERE, "-o", OPCOUNT_LIB + ".tmp", OPCOUNT_SRC]
        subprocess.check_call(cmd)
        os.replace(OPCOUNT_LIB + ".tmp", OPCOUNT_LIB)
    return OPCOUNT_LIB


def _opcount_lib():
    global _oplib
    if _oplib is None:
        stale = (not os.path.exists(OPCOUNT_LIB) or os.path.getmtime(OPCOUNT_LIB) < os.path.getmtime(SRC)
                 or os.path.getmtime(OPCOUNT_LIB) < os.path.getmtime(OPCOUNT_SRC))
        if stale:
            build_opcount()
        L = C.CDLL(OPCOUNT_LIB)
        dp = C.POINTER(C.c_double)
        L.og_face_flux.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp]
        L.og_face_flux.restype = C.c_int
        L.og_ops_reset.argtypes = []
        L.og_ops_get.argtypes = [C.POINTER(C.c_ulonglong)]
        _oplib = L
    return _oplib


def face_op_counts(dim, Wl, Wr, sl, sr, Wi, Wi1, dxl, dxr, kf, wf, Sf, dt, gamma=1.4, prandtl=0.72, mu=1e-3,
                   c_a=0.0, c_mu=0.09, eps_mode="dt"):
    """The oracle's operations for one face flux (the arguments of face_flux), by kind
    (OP_KINDS), from the counting build; also returns that build's flux."""
    L = _opcount_lib()
    nv = dim + 2
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (Wl, Wr, sl, sr)]
    wis = [np.ascontiguousarray(x, dtype=np.float64) for x in (Wi, Wi1)]
    params = np.array([gamma, prandtl, mu, c_a, c_mu, EPS_MODE[eps_mode]], dtype=np.float64)
    F, G, q, info = np.zeros(nv), np.zeros(nv), np.zeros(1), np.zeros(INFO_LEN)
    L.og_ops_reset()
    st = L.og_face_flux(dim, _dp(params), *[_dp(a) for a in arrs], None, None, *[_dp(a) for a in wis],
                        float(dxl), float(dxr), float(kf), float(wf), float(Sf), float(dt),
                        _dp(F), _dp(G), _dp(q), _dp(info))
    if st:
        raise OracleError(st)
    out = (C.c_ulonglong * len(OP_KINDS))()
    L.og_ops_get(out)
    return dict(zip(OP_KINDS, [int(v) for v in out])), F


def moments_u(U, lam):
    out = np.zeros(3 * NU)
    lib().og_moments_u(float(U), float(lam), _dp(out))
    return out.reshape(3, NU)


def kogan(tau, dt):
    out = np.zeros(9)
    lib().og_kogan(float(tau), float(dt), _dp(out))
    return out


def reconstruct(recon, w, xc, xf):
    """One component at one face between cells i and i+1: values w of cells i-1..i+2
    (i-2..i+3 for "weno5"), centres xc of cells i-1..i+2, face xf.  Returns (wl, wr, sl, sr)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    if w.shape != ((6,) if recon == "weno5" else (4,)):
        raise ValueError("reconstruct: wrong number of cell values")
    out = np.zeros(4)
    st = lib().og_recon(RECON[recon], _dp(w), _dp(np.ascontiguousarray(xc, dtype=np.float64)), float(xf), _dp(out))
    if st:
        raise OracleError(st)
    return tuple(out)


def weno5(v):
    """Fifth-order WENO value at the face between the third and fourth of five cell
    averages v (upwind side first)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    if v.shape != (5,):
        raise ValueError("weno5: five cell averages")
    return float(lib().og_weno5_value(_dp(v)))


def kogan_e(tau, tau_e, dt):
    """Time weights with decay time tau_e in the exponentials (the tau_hat mode)."""
    out = np.zeros(9)
    lib().og_kogan_e(float(tau), float(tau_e), float(dt), _dp(out))
    return out


def eps_field(case, W=None, k=None, omega=None):
    """eps_hat = tau/tau_hat of every face at the state's CFL step, largest per cell."""
    b = _Bound(case)
    out = np.zeros(case.ncells)
    st = lib().og_eps_field(b.ptr, _dp(_flat(case.W if W is None else W)), _dp(_flat(case.k if k is None else k)),
                            _dp(_flat(case.omega if omega is None else omega)), _dp(out))
    if st:
        raise OracleError(st)
    return out.reshape(case.k.shape)


def tau_field(case, W=None, k=None, omega=None):
    """The relaxation time tau of every face at the state's CFL step, largest per cell."""
    b = _Bound(case)
    out = np.zeros(case.ncells)
    st = lib().og_tau_field(b.ptr, _dp(_flat(case.W if W is None else W)), _dp(_flat(case.k if k is None else k)),
                            _dp(_flat(case.omega if omega is None else omega)), _dp(out))
    if st:
        raise OracleError(st)
    return out.reshape(case.k.shape)


def moment_solve(dim, gamma, rho, U, lam, r):
    p = np.array([rho, U[0], U[1] if len(U) > 1 else 0.0, U[2] if len(U) > 2 else 0.0, lam])
    r = np.ascontiguousarray(r, dtype=np.float64)
    x = np.zeros(dim + 2)
    st = lib().og_moment_solve(dim, float(gamma), _dp(p), _dp(r), _dp(x))
    if st:
        raise OracleError(st)
    return x


def tau_value(mu, c_a, c_mu, rho0, p0, pl, pr, kf, wf, Sf, dt):
    return lib().og_tau_value(mu, c_a, c_mu, rho0, p0, pl, pr, kf, wf, Sf, dt)
