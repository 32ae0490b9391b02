"""Exact solution of the 1D Riemann problem for an ideal gas (pressure-function method:
shock branch from the Rankine-Hugoniot relations, rarefaction branch from the isentropic
Riemann invariants; Newton iteration on p*).  Used to check the oracle on shock tubes."""
import math

import numpy as np


def _f(p, rho, pk, gamma):
    a = math.sqrt(gamma * pk / rho)
    if p > pk:   # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    r = p / pk
    return (2.0 * a / (gamma - 1.0) * (r ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0),
            1.0 / (rho * a) * r ** (-(gamma + 1.0) / (2.0 * gamma)))


def star_state(left, right, gamma=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dl = _f(p, rl, pl, gamma)
        fr, dr = _f(p, rr, pr, gamma)
        dp = (fl + fr + ur - ul) / (dl + dr)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-15 * p:
            break
    fl, _ = _f(p, rl, pl, gamma)
    fr, _ = _f(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)

    def rho_star(rho, pk):
        if p > pk:
            g = (gamma - 1.0) / (gamma + 1.0)
            return rho * (p / pk + g) / (g * p / pk + 1.0)
        return rho * (p / pk) ** (1.0 / gamma)

    return p, u, rho_star(rl, pl), rho_star(rr, pr)


def sample(left, right, x, t, x0=0.5, gamma=1.4):
    """(rho, u, p) at positions x and time t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us, rsl, rsr = star_state(left, right, gamma)
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    out = np.zeros((3, len(x)))
    for i, xi in enumerate(x):
        s = (xi - x0) / t
        if s <= us:   # left of contact
            if ps > pl:
                sh = ul - al * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                st = (rl, ul, pl) if s < sh else (rsl, us, ps)
            else:
                ast = al * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                head, tail = ul - al, us - ast
                if s < head:
                    st = (rl, ul, pl)
                elif s > tail:
                    st = (rsl, us, ps)
                else:
                    c = 2 / (gamma + 1) + (gamma - 1) / ((gamma + 1) * al) * (ul - s)
                    u = 2 / (gamma + 1) * (al + (gamma - 1) / 2 * ul + s)
                    st = (rl * c ** (2 / (gamma - 1)), u, pl * c ** (2 * gamma / (gamma - 1)))
        else:
            if ps > pr:
                sh = ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                st = (rr, ur, pr) if s > sh else (rsr, us, ps)
            else:
                ast = ar * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                head, tail = ur + ar, us + ast
                if s > head:
                    st = (rr, ur, pr)
                elif s < tail:
                    st = (rsr, us, ps)
                else:
                    c = 2 / (gamma + 1) - (gamma - 1) / ((gamma + 1) * ar) * (ur - s)
                    u = 2 / (gamma + 1) * (-ar + (gamma - 1) / 2 * ur + s)
                    st = (rr * c ** (2 / (gamma - 1)), u, pr * c ** (2 * gamma / (gamma - 1)))
        out[:, i] = st
    return out
