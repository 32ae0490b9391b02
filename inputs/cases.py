"""Case generators: grids, initial conservative states, boundary data, k and omega.

Every array is float64.  Conservative state W has shape (nvar, nz, ny, nx), x
fastest, nvar = dim + 2 (rho, rho*U, rho*V, [rho*W], rho*E).  In 2D nz = 1.
k and omega have shape (nz, ny, nx).  Face coordinates xf[d] hold n[d]+1 values.

The recipes stand in for the paper's wind-tunnel cases (whose geometries and
measured data are not reproduced): a periodic mixing layer, a wall-bounded
shock/boundary-layer interaction on a wall-stretched grid, a decaying isotropic
box, shock tubes, and small analytic flows used as checks.  All quantities are
nondimensional.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BC_NAMES = ("periodic", "wall", "dirichlet", "profile", "outflow")
C_MU = 0.09


def nvar_of(dim: int) -> int:
    return dim + 2


@dataclasses.dataclass
class Case:
    name: str
    dim: int
    n: tuple                      # (nx, ny, nz); nz == 1 in 2D
    xf: list                      # dim arrays of face coordinates
    bc: list                      # dim pairs of names from BC_NAMES
    bc_data: list                 # dim pairs of None | ndarray
    W: np.ndarray                 # (nvar, nz, ny, nx)
    k: np.ndarray                 # (nz, ny, nx)
    omega: np.ndarray             # (nz, ny, nx)
    gamma: float = 1.4
    prandtl: float = 0.72
    mu: float = 1e-3
    c_a: float = 0.0
    c_mu: float = C_MU
    cfl: float = 0.5
    t_end: float = 0.0            # 0 => no end time
    steps: int = 100
    precision: str = "fp64"       # "fp64" | "fp32_flux"
    max_steps: int = 0            # > 0: a solver stops after this many steps
    res_tol: float = 0.0          # > 0: a solver stops once max_m res_m / res_first_m <= res_tol
    kw_transport: bool = False    # transport k and omega with the flow (else frozen inputs)
    eps_mode: str = "dt"          # rarefaction in the time weights: "dt" (tau/dt) or "tauhat" (tau/tau_hat)
    recon: str = "muscl2"         # face values: "muscl2" (minmod), "muscl3" (limited kappa = 1/3) or "weno5"
    multi_d: bool = False         # expand the distributions along the tangential axes too
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nvar(self) -> int:
        return nvar_of(self.dim)

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def copy(self) -> "Case":
        c = dataclasses.replace(self)
        c.W = self.W.copy()
        c.k = self.k.copy()
        c.omega = self.omega.copy()
        c.xf = [a.copy() for a in self.xf]
        c.bc = [list(p) for p in self.bc]
        c.bc_data = [[None if a is None else np.array(a, copy=True) for a in p] for p in self.bc_data]
        c.meta = dict(self.meta)
        return c

    # scalar fields written to the case file (the arrays go to the .npz beside it)
    _SCALARS = ("name", "dim", "gamma", "prandtl", "mu", "c_a", "c_mu", "cfl", "t_end", "steps", "precision",
                "max_steps", "res_tol", "kw_transport", "eps_mode", "recon", "multi_d")

    def save(self, path: str) -> None:
        """Write the case as `path` (JSON: sizes, boundary names, gas and run parameters,
        options, meta) and `path` + ".npz" (the arrays: W, k, omega, face coordinates,
        boundary data); `Case.load(path)` reads it back bitwise."""
        import json
        doc = {f: getattr(self, f) for f in self._SCALARS}
        doc["n"] = [int(v) for v in self.n]
        doc["bc"] = [list(p) for p in self.bc]
        doc["bc_data"] = [[a is not None for a in p] for p in self.bc_data]
        doc["meta"] = {k: v for k, v in self.meta.items() if isinstance(v, (bool, int, float, str))}
        arrays = {"W": self.W, "k": self.k, "omega": self.omega}
        for d in range(self.dim):
            arrays[f"xf{d}"] = self.xf[d]
            for s in range(2):
                if self.bc_data[d][s] is not None:
                    arrays[f"bc{d}{s}"] = np.asarray(self.bc_data[d][s])
        with open(path, "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)
        np.savez(path + ".npz", **arrays)

    @classmethod
    def load(cls, path: str) -> "Case":
        """Read a case written by `save` (JSON and arrays only: nothing in the files is run)."""
        import json
        with open(path) as f:
            doc = json.load(f)
        with np.load(path + ".npz", allow_pickle=False) as z:
            a = {k: z[k] for k in z.files}
        dim = int(doc["dim"])
        bcd = [[a[f"bc{d}{s}"] if doc["bc_data"][d][s] else None for s in range(2)] for d in range(dim)]
        kw = {f: doc[f] for f in cls._SCALARS}
        return cls(n=tuple(doc["n"]), xf=[a[f"xf{d}"] for d in range(dim)], bc=doc["bc"], bc_data=bcd,
                   W=a["W"], k=a["k"], omega=a["omega"], meta=doc["meta"], **kw)


def cons_from_prim(rho, vel, p, gamma):
    """(rho, [U, V, (W)], p) -> conservative stack (nvar, ...)."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.asarray(v, dtype=np.float64) for v in vel]
    ke = 0.5 * rho * sum(v * v for v in vel)
    out = [rho] + [rho * v for v in vel] + [np.asarray(p, dtype=np.float64) / (gamma - 1.0) + ke]
    shape = np.broadcast_shapes(*[np.shape(a) for a in out])
    return np.stack([np.broadcast_to(a, shape) for a in out]).astype(np.float64)


def _uniform_faces(n, lo=0.0, hi=1.0):
    return np.linspace(lo, hi, n + 1, dtype=np.float64)


def _centres(xf):
    return 0.5 * (xf[1:] + xf[:-1])


def _omega_mixing(k, ell, c_mu=C_MU):
    return np.sqrt(k) / (c_mu ** 0.25 * ell)


# --------------------------------------------------------------------------
# Config: periodic double shear (mixing) layer
# --------------------------------------------------------------------------
def mixing_layer(N: int = 64, Ma: float = 0.3, seed: int = 0, gamma: float = 1.4,
                 mu: float = 1e-3, steps: int = 100, precision: str = "fp64",
                 ny: Optional[int] = None) -> Case:
    """2D periodic double shear layer on [0,1)^2, tanh profile + seeded noise."""
    nx, ny = N, (N if ny is None else ny)
    xf, yf = _uniform_faces(nx), _uniform_faces(ny)
    x, y = _centres(xf), _centres(yf)
    Y, X = np.meshgrid(y, x, indexing="ij")
    delta = 0.04
    Uinf = 1.0
    rng = np.random.default_rng(seed)
    U = Uinf * (np.tanh((Y - 0.25) / delta) - np.tanh((Y - 0.75) / delta) - 1.0)
    V = np.zeros_like(U)
    U = U + 1e-3 * Uinf * rng.uniform(-1.0, 1.0, size=U.shape)
    V = V + 1e-3 * Uinf * rng.uniform(-1.0, 1.0, size=V.shape)
    rho = np.ones_like(U)
    p = np.full_like(U, 1.0 / (gamma * Ma * Ma))
    W = cons_from_prim(rho, [U, V], p, gamma)[:, None, :, :]
    k = 1e-3 * Uinf ** 2 * (np.exp(-((Y - 0.25) / delta) ** 2) + np.exp(-((Y - 0.75) / delta) ** 2))
    k = np.maximum(k, 1e-12)
    omega = _omega_mixing(k, 0.14 * delta)
    return Case(
        name=f"mixing_layer_{nx}x{ny}", dim=2, n=(nx, ny, 1), xf=[xf, yf],
        bc=[["periodic", "periodic"], ["periodic", "periodic"]],
        bc_data=[[None, None], [None, None]],
        W=np.ascontiguousarray(W), k=k[None].copy(), omega=omega[None].copy(),
        gamma=gamma, prandtl=0.72, mu=mu, c_a=0.0, cfl=0.5, steps=steps,
        precision=precision, meta={"Ma": Ma, "seed": seed, "delta": delta},
    )


# --------------------------------------------------------------------------
# Config: shock / turbulent boundary-layer interaction on a stretched grid
# --------------------------------------------------------------------------
def oblique_shock(M1: float, theta_deg: float, gamma: float = 1.4):
    """Weak-branch oblique shock: returns (beta_rad, p2/p1, rho2/rho1, Vt, Vn ratio).

    Solves tan(theta) = 2 cot(beta) (M^2 sin^2 beta - 1) / (M^2 (gamma + cos 2beta) + 2)
    by bisection on the weak branch.
    """
    th = math.radians(theta_deg)

    def f(b):
        return 2.0 / math.tan(b) * (M1 * M1 * math.sin(b) ** 2 - 1.0) / (
            M1 * M1 * (gamma + math.cos(2 * b)) + 2.0) - math.tan(th)

    mu_angle = math.asin(1.0 / M1)
    # weak branch lies between the Mach angle and the max-deflection angle
    bs = np.linspace(mu_angle + 1e-9, math.pi / 2 - 1e-9, 20001)
    vals = np.array([f(b) for b in bs])
    i = int(np.argmax(vals > 0))
    lo, hi = bs[i - 1], bs[i]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    beta = 0.5 * (lo + hi)
    mn1 = M1 * math.sin(beta)
    p21 = 1.0 + 2.0 * gamma / (gamma + 1.0) * (mn1 * mn1 - 1.0)
    r21 = (gamma + 1.0) * mn1 * mn1 / ((gamma - 1.0) * mn1 * mn1 + 2.0)
    return beta, p21, r21


def sbli(nx: int = 1024, ny: int = 512, seed: int = 1, gamma: float = 1.4,
         mu: float = 1e-5, steps: int = 2000, precision: str = "fp64",
         stretch: float = 3.0) -> Case:
    """Mach-2 flow over an adiabatic no-slip wall hit by an 8-degree oblique shock.

    Domain [0,2]x[0,1]; uniform in x, tanh wall stretching in y.  Left: fixed
    inflow; right: zeroth-order outflow; bottom: no-slip adiabatic wall; top:
    a fixed profile that is freestream upstream of the shock foot and the
    post-shock state beyond it, placed so the inviscid impingement is x = 1.5.
    """
    M = 2.0
    rho1, u1, p1 = 1.0, 1.0, 1.0 / (gamma * M * M)
    xf = _uniform_faces(nx, 0.0, 2.0)
    eta = np.linspace(0.0, 1.0, ny + 1)
    yf = 1.0 - np.tanh(stretch * (1.0 - eta)) / math.tanh(stretch)
    yf[0], yf[-1] = 0.0, 1.0
    x, y = _centres(xf), _centres(yf)
    beta, p21, r21 = oblique_shock(M, 8.0, gamma)
    th = math.radians(8.0)
    ut = u1 * math.cos(beta)
    un2 = u1 * math.sin(beta) / r21
    speed2 = math.hypot(ut, un2)
    u2, v2 = speed2 * math.cos(th), -speed2 * math.sin(th)
    rho2, p2 = rho1 * r21, p1 * p21
    x_foot = 1.5 - 1.0 / math.tan(beta)
    free = cons_from_prim(rho1, [u1, 0.0], p1, gamma)
    post = cons_from_prim(rho2, [u2, v2], p2, gamma)
    prof = np.where(x[None, :] < x_foot, free[:, None], post[:, None]).astype(np.float64)
    Y, X = np.meshgrid(y, x, indexing="ij")
    W = np.broadcast_to(free[:, None, None, None], (4, 1, ny, nx)).copy()
    rng = np.random.default_rng(seed)
    dbl = 0.05
    k = 5e-3 * u1 ** 2 * (Y / dbl) * np.exp(1.0 - Y / dbl) * (1.0 + 0.05 * rng.uniform(-1, 1, size=Y.shape))
    k = np.maximum(k, 0.0)
    ell = np.maximum(np.minimum(0.41 * Y, 0.09 * dbl), 1e-6)
    omega = np.sqrt(np.maximum(k, 1e-30)) / (C_MU ** 0.25 * ell)
    return Case(
        name=f"sbli_{nx}x{ny}", dim=2, n=(nx, ny, 1), xf=[xf, yf],
        bc=[["dirichlet", "outflow"], ["wall", "profile"]],
        bc_data=[[free.copy(), None], [None, np.ascontiguousarray(prof)]],
        W=W, k=k[None].copy(), omega=omega[None].copy(),
        gamma=gamma, prandtl=0.72, mu=mu, c_a=0.0, cfl=0.5, steps=steps,
        precision=precision,
        meta={"seed": seed, "beta_deg": math.degrees(beta), "x_foot": x_foot,
              "post_shock": (rho2, u2, v2, p2)},
    )


# --------------------------------------------------------------------------
# Config: decaying isotropic turbulence in a periodic box
# --------------------------------------------------------------------------
def isotropic_box(N: int = 256, seed: int = 2, Ma_t: float = 0.5, k0: float = 4.0,
                  gamma: float = 1.4, mu: float = 1e-3, steps: int = 500,
                  precision: str = "fp32_flux") -> Case:
    """[0,2pi)^3 periodic box, random-phase solenoidal field, E ~ k^4 exp(-2 (k/k0)^2)."""
    rng = np.random.default_rng(seed)
    L = 2.0 * math.pi
    f = _uniform_faces(N, 0.0, L)
    kk = np.fft.fftfreq(N, d=1.0 / N)
    kr = np.fft.rfftfreq(N, d=1.0 / N)
    KZ, KY, KX = np.meshgrid(kk, kk, kr, indexing="ij")   # array index (z, y, x)
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    Kmag = np.sqrt(K2)
    E = Kmag ** 4 * np.exp(-2.0 * (Kmag / k0) ** 2)
    amp = np.zeros_like(Kmag)
    nz = Kmag > 0
    amp[nz] = np.sqrt(E[nz] / (4.0 * math.pi * K2[nz]))
    comps = []
    for _ in range(3):
        noise = rng.standard_normal((N, N, N))
        comps.append(np.fft.rfftn(noise) * amp)
    ux_h, uy_h, uz_h = comps
    # solenoidal projection
    dot = np.zeros_like(ux_h)
    K2s = np.where(K2 > 0, K2, 1.0)
    dot = (KX * ux_h + KY * uy_h + KZ * uz_h) / K2s
    ux_h = ux_h - KX * dot
    uy_h = uy_h - KY * dot
    uz_h = uz_h - KZ * dot
    ax = (0, 1, 2)
    ux = np.fft.irfftn(ux_h, s=(N, N, N), axes=ax)
    uy = np.fft.irfftn(uy_h, s=(N, N, N), axes=ax)
    uz = np.fft.irfftn(uz_h, s=(N, N, N), axes=ax)
    rms = math.sqrt(float(np.mean(ux ** 2 + uy ** 2 + uz ** 2)))
    s = Ma_t / rms
    ux, uy, uz = ux * s, uy * s, uz * s
    # resolved dissipation from spectral gradients
    grad2 = 0.0
    for comp in (ux, uy, uz):
        ch = np.fft.rfftn(comp)
        for Kd in (KX, KY, KZ):
            g = np.fft.irfftn(1j * Kd * ch, s=(N, N, N), axes=ax)
            grad2 += float(np.mean(g * g))
    nu = mu / 1.0
    K_res = 0.5 * float(np.mean(ux ** 2 + uy ** 2 + uz ** 2))
    eps_res = nu * grad2
    kt = 0.1 * K_res
    om = eps_res / (C_MU * K_res)
    rho = np.ones_like(ux)
    p = np.full_like(ux, 1.0 / gamma)
    W = cons_from_prim(rho, [ux, uy, uz], p, gamma)
    return Case(
        name=f"isotropic_{N}^3", dim=3, n=(N, N, N), xf=[f, f.copy(), f.copy()],
        bc=[["periodic", "periodic"]] * 3, bc_data=[[None, None]] * 3,
        W=np.ascontiguousarray(W), k=np.full((N, N, N), kt), omega=np.full((N, N, N), om),
        gamma=gamma, prandtl=0.72, mu=mu, c_a=0.0, cfl=0.5, steps=steps,
        precision=precision, meta={"seed": seed, "K_res": K_res, "eps_res": eps_res},
    )


# --------------------------------------------------------------------------
# Shock tubes
# --------------------------------------------------------------------------
def shock_tube(nx: int, ny: int = 4, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1),
               x0: float = 0.5, shift: float = 0.0, gamma: float = 1.4, mu: float = 0.0,
               c_a: float = 1.0, k_val: float = 0.0, omega_val: float = 1.0,
               t_end: float = 0.0, steps: int = 100000, precision: str = "fp64",
               bc_x=("outflow", "outflow"), name: str = "shock_tube") -> Case:
    """Riemann problem along x on [0,1] x [0, ny/nx], periodic in y.

    `shift` adds a uniform x-velocity to both states (Galilean shift)."""
    xf = _uniform_faces(nx)
    yf = _uniform_faces(ny, 0.0, ny / nx)
    x = _centres(xf)
    rl, ul, pl = left
    rr, ur, pr = right
    rho = np.where(x < x0, rl, rr)
    u = np.where(x < x0, ul, ur) + shift
    p = np.where(x < x0, pl, pr)
    W1 = cons_from_prim(rho, [u, np.zeros_like(u)], p, gamma)     # (4, nx)
    W = np.broadcast_to(W1[:, None, None, :], (4, 1, ny, nx)).copy()
    bcd = [[None, None], [None, None]]
    if bc_x[0] == "dirichlet":
        bcd[0][0] = cons_from_prim(rl, [ul + shift, 0.0], pl, gamma)
    if bc_x[1] == "dirichlet":
        bcd[0][1] = cons_from_prim(rr, [ur + shift, 0.0], pr, gamma)
    return Case(
        name=f"{name}_{nx}x{ny}", dim=2, n=(nx, ny, 1), xf=[xf, yf],
        bc=[list(bc_x), ["periodic", "periodic"]], bc_data=bcd, W=W,
        k=np.full((1, ny, nx), k_val), omega=np.full((1, ny, nx), omega_val),
        gamma=gamma, prandtl=1.0, mu=mu, c_a=c_a, cfl=0.5, t_end=t_end, steps=steps,
        precision=precision, meta={"x0": x0, "shift": shift, "left": left, "right": right},
    )


def sod_tube(nx: int = 100, ny: int = 2, t_end: float = 0.2, **kw) -> Case:
    """Sod's problem (1,0,1 | 0.125,0,0.1), gamma 1.4, diaphragm at 0.5."""
    return shock_tube(nx, ny, t_end=t_end, name="sod", **kw)


# --------------------------------------------------------------------------
# Analytic check flows
# --------------------------------------------------------------------------
def shear_wave(N: int = 64, amp_over_c: float = 1e-4, mu: float = 1e-2, k_val: float = 0.0,
               omega_val: float = 1.0, gamma: float = 1.4, steps: int = 100) -> Case:
    """U = A sin(2 pi y), uniform rho=1, p=1/gamma (c=1), periodic unit square."""
    xf, yf = _uniform_faces(N), _uniform_faces(N)
    x, y = _centres(xf), _centres(yf)
    Y, X = np.meshgrid(y, x, indexing="ij")
    A = amp_over_c * 1.0
    U = A * np.sin(2 * math.pi * Y)
    W = cons_from_prim(np.ones_like(U), [U, np.zeros_like(U)], np.full_like(U, 1.0 / gamma), gamma)
    return Case(
        name=f"shear_wave_{N}", dim=2, n=(N, N, 1), xf=[xf, yf],
        bc=[["periodic", "periodic"]] * 2, bc_data=[[None, None]] * 2,
        W=W[:, None].copy(), k=np.full((1, N, N), k_val), omega=np.full((1, N, N), omega_val),
        gamma=gamma, prandtl=0.72, mu=mu, c_a=0.0, cfl=0.5, steps=steps,
        meta={"A": A},
    )


def entropy_wave(N: int = 64, ny: int = 2, U: float = 1.0, amp: float = 0.2,
                 gamma: float = 1.4, t_end: float = 1.0) -> Case:
    """rho = 1 + amp sin(2 pi x), uniform U and p: advected exactly by the Euler equations."""
    xf = _uniform_faces(N)
    yf = _uniform_faces(ny, 0.0, ny / N)
    x = _centres(xf)
    # cell averages of 1 + amp sin(2 pi x)
    dx = xf[1:] - xf[:-1]
    rho1 = 1.0 - amp * (np.cos(2 * math.pi * xf[1:]) - np.cos(2 * math.pi * xf[:-1])) / (2 * math.pi * dx)
    rho = np.broadcast_to(rho1[None, :], (ny, N))
    W = cons_from_prim(rho, [np.full_like(rho, U), np.zeros_like(rho)], np.ones_like(rho), gamma)
    return Case(
        name=f"entropy_wave_{N}", dim=2, n=(N, ny, 1), xf=[xf, yf],
        bc=[["periodic", "periodic"]] * 2, bc_data=[[None, None]] * 2,
        W=W[:, None].copy(), k=np.zeros((1, ny, N)), omega=np.ones((1, ny, N)),
        gamma=gamma, prandtl=1.0, mu=0.0, c_a=0.0, cfl=0.5, t_end=t_end, steps=10 ** 7,
        meta={"U": U, "amp": amp},
    )


def uniform_flow(dim: int = 2, n=(16, 12, 1), rho=1.3, vel=(0.7, -0.4, 0.2), p=0.9,
                 stretched: bool = True, seed: int = 5, gamma: float = 1.4, mu: float = 1e-3,
                 bc=None) -> Case:
    """Uniform state on a (randomly) stretched grid with random positive k/omega fields."""
    rng = np.random.default_rng(seed)
    xf = []
    for d in range(dim):
        nd = n[d]
        if stretched:
            w = rng.uniform(0.5, 2.0, size=nd)
            f = np.concatenate([[0.0], np.cumsum(w)]) / w.sum()
        else:
            f = _uniform_faces(nd)
        xf.append(f.astype(np.float64))
    shape = (n[2], n[1], n[0]) if dim == 3 else (1, n[1], n[0])
    vel = list(vel[:dim])
    W0 = cons_from_prim(rho, vel, p, gamma)
    W = np.broadcast_to(W0.reshape(-1, 1, 1, 1), (dim + 2,) + shape).copy()
    k = rng.uniform(0.0, 1e-2, size=shape)
    om = rng.uniform(1.0, 10.0, size=shape)
    if bc is None:
        bc = [["periodic", "periodic"]] * dim
    bcd = [[None, None] for _ in range(dim)]
    for d in range(dim):
        for s in range(2):
            if bc[d][s] == "dirichlet":
                bcd[d][s] = W0.copy()
            elif bc[d][s] == "profile":
                ntan = int(np.prod([n[a] for a in range(dim) if a != d]))
                bcd[d][s] = np.repeat(W0[:, None], ntan, axis=1).copy()
    nn = (n[0], n[1], n[2] if dim == 3 else 1)
    return Case(
        name=f"uniform_{dim}d", dim=dim, n=nn, xf=xf, bc=[list(p_) for p_ in bc], bc_data=bcd,
        W=W, k=k, omega=om, gamma=gamma, prandtl=0.72, mu=mu, c_a=0.0, cfl=0.5, steps=5,
    )


# --------------------------------------------------------------------------
# Batched and served workloads
# --------------------------------------------------------------------------
def batch_cases(count: int = 64, seed: int = 3, nmin: int = 64, nmax: int = 512,
                steps: int = 200, precision: str = "fp32_flux") -> List[Case]:
    """Uneven batch: square 2D mixing layers and Galilean-shifted Sod tubes."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(rng.integers(nmin, nmax + 1))
        Ma = float(rng.uniform(0.2, 2.0))
        kind = int(rng.integers(0, 2))
        if kind == 0:
            c = mixing_layer(N, Ma=Ma, seed=int(rng.integers(0, 2 ** 31)), steps=steps,
                             precision=precision)
        else:
            gamma = 1.4
            ub = Ma * math.sqrt(gamma * 1.0 / 1.0)
            c = shock_tube(N, N, x0=0.25, shift=ub, mu=1e-4, c_a=1.0, k_val=1e-6, omega_val=10.0,
                           steps=steps, precision=precision, bc_x=("dirichlet", "outflow"),
                           name="shifted_sod")
        c.name = f"b{i:02d}_{c.name}"
        c.meta["batch_index"] = i
        out.append(c)
    return out


def serve_trace(count: int = 256, seed: int = 4, rate: float = 20.0,
                n2d=(128, 1024), n3d=(64, 128), max_steps: int = 5000,
                tol: float = 1e-6):
    """Poisson arrivals; each request names a family and a size, built lazily."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        fam = int(rng.integers(0, 3))
        if fam == 2:
            side = int(rng.integers(n3d[0], n3d[1] + 1))
        else:
            side = int(rng.integers(n2d[0], n2d[1] + 1))
        reqs.append({"id": i, "arrival": t, "family": fam, "side": side,
                     "seed": int(rng.integers(0, 2 ** 31)), "max_steps": max_steps, "tol": tol})
    return reqs


def request_case(req) -> Case:
    """Materialise one served request (family 0: mixing layer FP64; 1: SBLI FP32-flux;
    2: isotropic box FP32-flux)."""
    fam, side, seed = req["family"], req["side"], req["seed"]
    if fam == 0:
        c = mixing_layer(side, seed=seed, steps=req["max_steps"], precision="fp64")
    elif fam == 1:
        c = sbli(side, max(side // 2, 8), seed=seed, steps=req["max_steps"], precision="fp32_flux")
    else:
        c = isotropic_box(side, seed=seed, steps=req["max_steps"], precision="fp32_flux")
    c.name = f"req{req['id']}_{c.name}"
    c.max_steps = int(req["max_steps"])
    c.res_tol = float(req["tol"])
    return c


def config_case(index: int, scale: Optional[int] = None) -> Case:
    """The benchmark configurations by index (0: mixing layer 64^2, 1: SBLI 1024x512,
    2: isotropic 256^3).  `scale` shrinks the grid for parity runs."""
    if index == 0:
        return mixing_layer(64 if scale is None else scale)
    if index == 1:
        if scale is None:
            return sbli()
        return sbli(scale, max(scale // 2, 8))
    if index == 2:
        return isotropic_box(256 if scale is None else scale)
    raise ValueError(index)
