"""The flux kernel's time weights of the Kogan solution (gam0..gam5 and the ratios c1, c4,
c5) against their closed forms in 60-digit mpmath, on both sides of the switch from the
power series (x = dt/tau < 1/2) to the exponential form.

Bounds: in the series branch every weight is a product of well-conditioned factors, so a
few ulp; in the exponential branch the combinations cancel, and the bound is a few ulp
times the ratio of the largest term to the result (condition number of the formula)."""
import os
import subprocess

import mpmath
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = r"""
#include <cmath>
#include <cstdio>
#define GKS_HD
#include "gks_flux.hpp"
int main() {
    double tau, dt;
    while (std::scanf("%lf %lf", &tau, &dt) == 2) {
        const gks::Kw<double> k = gks::kogan(tau, dt);
        const gks::Kw<float> f = gks::kogan((float)tau, (float)dt);
        for (int i = 0; i < 6; ++i) std::printf("%.17g ", k.g[i]);
        std::printf("%.17g %.17g %.17g ", k.c1, k.c4, k.c5);
        for (int i = 0; i < 6; ++i) std::printf("%.9g ", (double)f.g[i]);
        std::printf("%.9g %.9g %.9g\n", (double)f.c1, (double)f.c4, (double)f.c5);
    }
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("kogan")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    exe = d / "h"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I",
                           os.path.join(ROOT, "paper_1302_2132_amd", "csrc"), "-o", str(exe), str(src)])
    return str(exe)


def _exact(tau, dt):
    """Closed forms of the weights (the definitions, not the kernel's rearrangement)."""
    t, h = mpmath.mpf(tau), mpmath.mpf(dt)
    E = mpmath.exp(-h / t)
    g = [h - t * (1 - E),
         2 * t * t * (1 - E) - t * h * (1 + E),
         h * h / 2 - t * h + t * t * (1 - E),
         t * (1 - E),
         -(2 * t * t * (1 - E) - t * h * E),
         -t * t * (1 - E)]
    c = [g[1] / (t * g[0]), g[4] / (t * g[0]), g[5] / (t * g[0])]
    return g + c


def _cond(x):
    """Condition numbers of the exponential-branch formulas (largest term over result)."""
    E = np.exp(-x)
    s = 1 - E
    g0 = x - s
    g1 = 2 * s - x * (1 + E)
    g2 = 0.5 * x * x - x + s
    g4 = 2 * s - x * E
    c0 = x / abs(g0)
    c1 = max(2 * s, x * (1 + E)) / abs(g1)
    c2 = max(0.5 * x * x, x) / abs(g2)
    c4 = max(2 * s, x * E) / abs(g4)
    return np.array([c0 + 1, c1 + c0, c2 + 1, 1, c4 + 1, 1, c1 + c0, c4 + c0, c0 + 1])


def test_kogan_weights_fp64_and_fp32(harness):
    mpmath.mp.dps = 60
    dt = 1e-3
    xs = np.concatenate([np.geomspace(1e-8, 0.4999, 120), [0.5, 0.50001], np.geomspace(0.5001, 60, 80)])
    taus = dt / xs
    inp = "\n".join(f"{float(t)!r} {dt!r}" for t in taus)
    out = subprocess.run([harness], input=inp, capture_output=True, text=True, check=True).stdout
    v = np.array([[float(w) for w in line.split()] for line in out.strip().splitlines()])
    d64, d32 = v[:, :9], v[:, 9:]
    eps64, eps32 = 2.0 ** -53, 2.0 ** -24
    for i, (x, tau) in enumerate(zip(xs, taus)):
        ex = np.array([float(e) for e in _exact(tau, dt)])
        ex32 = np.array([float(e) for e in _exact(float(np.float32(tau)), float(np.float32(dt)))])
        cond = np.ones(9) if x < 0.5 else _cond(x)
        rel = np.abs(d64[i] - ex) / np.abs(ex)
        assert np.all(rel < 16 * eps64 * cond), (x, rel, cond)
        rel32 = np.abs(d32[i] - ex32) / np.abs(ex32)
        assert np.all(rel32 < 16 * eps32 * cond), (x, rel32, cond)


def test_kogan_limit_tau_zero(harness):
    out = subprocess.run([harness], input="0.0 0.01", capture_output=True, text=True, check=True).stdout
    v = [float(w) for w in out.split()]
    assert v[:9] == [0.01, 0.0, 0.5 * 0.01 * 0.01, 0.0, 0.0, 0.0, -1.0, 0.0, 0.0]
