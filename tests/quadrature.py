"""Brute-force numerical integration over a Maxwellian, for pinning the oracle.

Nothing here uses a closed-form Gaussian moment: tangential velocities are
integrated with Gauss-Hermite nodes, the internal energy X = |xi|^2 (a Gamma
variable with shape K/2 and scale 1/lambda for K internal degrees of freedom)
with generalised Gauss-Laguerre nodes, and the normal velocity with Gauss-Hermite
over the whole line or composite Gauss-Legendre over a half line.
"""
import math

import numpy as np
from scipy.special import gammaln, roots_genlaguerre, roots_hermite, roots_legendre

_LEG = {}


def _leg(n):
    if n not in _LEG:
        _LEG[n] = roots_legendre(n)
    return _LEG[n]


def composite_legendre(a, b, nsub=16, n=40):
    x0, w0 = _leg(n)
    edges = np.linspace(a, b, nsub + 1)
    xs, ws = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        xs.append(0.5 * (hi - lo) * x0 + 0.5 * (hi + lo))
        ws.append(0.5 * (hi - lo) * w0)
    return np.concatenate(xs), np.concatenate(ws)


class Maxwell:
    """rho-weighted integrals  int phi(u, v, w, X) g dXi  over u in all / u>0 / u<0."""

    def __init__(self, rho, U, lam, K, dim, nh=30, nlag=16, nsub=24, nleg=40):
        self.rho, self.lam, self.K, self.dim = rho, lam, K, dim
        self.U = np.zeros(3)
        self.U[:dim] = U[:dim]
        s = 1.0 / math.sqrt(lam)
        th, wh = roots_hermite(nh)
        self.tan_nodes = []
        for d in range(1, 3):
            if d < dim:
                self.tan_nodes.append((self.U[d] + s * th, wh / math.sqrt(math.pi)))
            else:
                self.tan_nodes.append((np.zeros(1), np.ones(1)))
        if K > 0:
            a = K / 2.0 - 1.0
            y, wy = roots_genlaguerre(nlag, a)
            self.X = y / lam
            self.wX = wy / math.exp(gammaln(K / 2.0))
        else:
            self.X, self.wX = np.zeros(1), np.ones(1)
        self.u_all = (self.U[0] + s * th, wh / math.sqrt(math.pi))
        span = self.U[0] + 40.0 * s
        dens = lambda u: math.sqrt(lam / math.pi) * np.exp(-lam * (u - self.U[0]) ** 2)
        if span > 0:
            x, w = composite_legendre(0.0, span, nsub, nleg)
            self.u_pos = (x, w * dens(x))
        else:
            self.u_pos = (np.zeros(1), np.zeros(1))
        span = self.U[0] - 40.0 * s
        if span < 0:
            x, w = composite_legendre(span, 0.0, nsub, nleg)
            self.u_neg = (x, w * dens(x))
        else:
            self.u_neg = (np.zeros(1), np.zeros(1))

    def integrate(self, phi, rng="all"):
        """phi(u, v, w, X) -> array broadcast over a 4-D tensor grid (or a list of arrays)."""
        un, uw = {"all": self.u_all, "pos": self.u_pos, "neg": self.u_neg}[rng]
        (vn, vw), (wn, ww) = self.tan_nodes
        u = un[:, None, None, None]
        v = vn[None, :, None, None]
        w = wn[None, None, :, None]
        X = self.X[None, None, None, :]
        wt = uw[:, None, None, None] * vw[None, :, None, None] * ww[None, None, :, None] * self.wX[None, None, None, :]
        vals = phi(u, v, w, X)
        if isinstance(vals, (list, tuple)):
            return np.array([self.rho * float(np.sum(np.broadcast_to(x, wt.shape) * wt)) for x in vals])
        return self.rho * float(np.sum(np.broadcast_to(vals, wt.shape) * wt))


def psi_list(dim, u, v, w, X):
    """psi = (1, u, v, [w], (u^2 + v^2 + [w^2] + X)/2) in the face-local frame."""
    one = np.ones_like(u * v * w * X)
    vel = [u, v, w][:dim]
    e = 0.5 * (sum(c * c for c in vel) + X)
    return [one] + [c * one for c in vel] + [e * one]


def lin(a, dim, u, v, w, X):
    ps = psi_list(dim, u, v, w, X)
    return sum(a[m] * ps[m] for m in range(dim + 2))


def maxwell_from_cons(W, dim, gamma):
    rho = W[0]
    U = np.array(W[1:1 + dim]) / rho
    p = (gamma - 1.0) * (W[dim + 1] - 0.5 * rho * float(U @ U))
    b = 2.0 / (gamma - 1.0)
    return rho, U, rho / (2.0 * p), b - dim, p


def time_weights_quad(tau, dt, n=48):
    """Time integrals over [0, dt] of the six coefficient functions of the Kogan solution,
    by composite Gauss-Legendre with the integrands evaluated in 40-digit arithmetic
    (they cancel badly when tau >> dt)."""
    import mpmath
    mpmath.mp.dps = 40
    if tau > 0:
        cut = min(dt, 50.0 * tau)
        t1, w1 = composite_legendre(0.0, cut, 24, n)
        if cut < dt:
            t2, w2 = composite_legendre(cut, dt, 8, n)
            t1, w1 = np.concatenate([t1, t2]), np.concatenate([w1, w2])
    else:
        t1, w1 = composite_legendre(0.0, dt, 4, n)
    tau_m = mpmath.mpf(tau)
    sums = [mpmath.mpf(0)] * 6
    for t, w in zip(t1, w1):
        t = mpmath.mpf(t)
        E = mpmath.exp(-t / tau_m) if tau > 0 else mpmath.mpf(0)
        fs = (1 - E, -tau_m + tau_m * E + t * E, t - tau_m + tau_m * E, E, -(t + tau_m) * E, -tau_m * E)
        for i in range(6):
            sums[i] += fs[i] * w
    return np.array([float(x) for x in sums])
