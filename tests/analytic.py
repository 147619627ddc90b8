"""Closed-form solutions used to pin the oracle (test helper, no method code).

2-D acoustic Green's function: for (1/v^2) u_tt - Lap u = w(t) delta(x), the
causal solution at distance r is
    u(r, t) = (1/(2 pi)) int_{r/v}^{t} w(t - tau) / sqrt(tau^2 - r^2/v^2) d tau,
and the substitution tau = (r/v) cosh(theta) removes the singularity:
    u(r, t) = (1/(2 pi)) int_0^{acosh(v t / r)} w(t - (r/v) cosh theta) d theta.
The integral is evaluated with composite Gauss-Legendre quadrature.
"""
import math

import numpy as np


def ricker_causal(t, f0, t0):
    t = np.asarray(t, dtype=np.float64)
    a = (math.pi * f0 * (t - t0)) ** 2
    w = (1.0 - 2.0 * a) * np.exp(-a)
    return np.where(t >= 0.0, w, 0.0)


def green2d_ricker(r, v, f0, times, t0=None, panels=64, order=16):
    """u(r, t) for the 2-D wave equation driven by a causal Ricker wavelet."""
    if t0 is None:
        t0 = 1.0 / f0
    xg, wg = np.polynomial.legendre.leggauss(order)
    out = np.zeros(len(times))
    for k, t in enumerate(times):
        if v * t <= r:
            continue
        thmax = math.acosh(v * t / r)
        edges = np.linspace(0.0, thmax, panels + 1)
        s = 0.0
        for a, b in zip(edges[:-1], edges[1:]):
            th = 0.5 * (b - a) * xg + 0.5 * (b + a)
            s += 0.5 * (b - a) * float(np.sum(wg * ricker_causal(t - (r / v) * np.cosh(th), f0, t0)))
        out[k] = s / (2.0 * math.pi)
    return out
