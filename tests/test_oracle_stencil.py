"""Pins of the oracle's stencil weights, stability limit, Ricker wavelet and damping."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import fd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fornberg_table():
    rows = {}
    with open(os.path.join(GOLDEN, "fornberg_second_derivative.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            order, vals = line.split(":")
            rows[int(order)] = [Fraction(v) for v in vals.split()]
    return rows


@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_weights_match_published_table(M):
    assert fd.fd_weights(M) == _fornberg_table()[2 * M]


def test_weights_exact_on_polynomials():
    # sum_k c_|k| k^p = p(p-1) 0^(p-2): exact second derivative at 0 for p <= 9
    c = fd.fd_weights(4)
    for p in range(0, 10):
        s = sum(c[abs(k)] * Fraction(k) ** p for k in range(-4, 5))
        assert s == (2 if p == 2 else 0), p
    # and not exact at degree 10 (the order is exactly 8)
    s = sum(c[abs(k)] * Fraction(k) ** 10 for k in range(-4, 5))
    assert s != 0


def test_weights_spectral_accuracy_order():
    # sin(kx): stencil gives -k^2 (1 + O((kh)^8)); error ratio under halving h ~ 2^8
    c = [float(v) for v in fd.fd_weights(4)]
    errs = []
    for h in (0.4, 0.2):
        approx = (c[0] + 2 * sum(c[k] * math.cos(k * h) for k in range(1, 5))) / h ** 2
        errs.append(abs(approx + 1.0))
    assert math.log2(errs[0] / errs[1]) == pytest.approx(8.0, abs=0.1)


def test_symbol_at_pi_closed_form():
    c = fd.fd_weights(4)
    s = c[0] + 2 * sum(c[k] * (-1) ** k for k in range(1, 5))
    assert s == Fraction(-2048, 315)
    th = np.linspace(0, np.pi, 10001)
    sv = fd.symbol(c, th)
    assert np.argmax(np.abs(sv)) == len(th) - 1


def test_stable_dt_closed_form():
    for (v, dz, dx) in [(2700.0, 10.0, 10.0), (6000.0, 10.0, 10.0), (5500.0, 8.0, 25.0)]:
        exact = 2.0 / (v * math.sqrt(2048.0 / 315.0 * (1 / dz ** 2 + 1 / dx ** 2)))
        assert fd.stable_dt(v, dz, dx) == pytest.approx(exact, rel=1e-12)
    # Courant limit for equal spacing
    assert fd.stable_dt(1.0, 1.0, 1.0) == pytest.approx(0.554632, abs=1e-6)


@pytest.mark.parametrize("factor,grows", [(0.99, False), (1.01, True)])
def test_stability_limit_by_time_stepping(factor, grows):
    # Dirichlet box, no absorbing layer, random initial field, 10^4 steps
    n = 100
    v = 2000.0
    h = 10.0
    dt = factor * fd.stable_dt(v, h, h)
    rng = np.random.default_rng(0)
    u0 = rng.standard_normal((n, n))
    vel = np.full((n, n), v)
    damp = np.zeros((n, n))
    _, fin = fd.forward_run(vel, damp, h, h, dt, 10001, None, [], [], 0, u0=u0, um1=u0,
                            want_final=True)
    amp = np.max(np.abs(fin)) if np.all(np.isfinite(fin)) else np.inf
    if grows:
        assert amp > 1e6
    else:
        assert amp < 100.0


def test_ricker_properties():
    f0 = 10.0
    dt = 1e-5
    nt = 40001
    w = fd.ricker(f0, dt, nt)
    t = np.arange(nt) * dt
    t0 = 1.0 / f0
    k0 = int(round(t0 / dt))
    assert w[k0] == pytest.approx(1.0, abs=1e-12)
    assert np.argmax(w) == k0
    tz = t0 + 1.0 / (math.pi * f0 * math.sqrt(2.0))
    assert fd.ricker(f0, tz, 2)[1] == pytest.approx(0.0, abs=1e-14)
    # integral over the whole line is zero (tail before t=0 is ~1e-4 of the area scale)
    assert abs(np.sum(w) * dt) < 1e-5


def test_damping_profile_definition():
    nz, nx, nbl, h, vmax, R = 20, 30, 10, 10.0, 3000.0, 1e-3
    d = fd.damping_profile(nz, nx, nbl, h, h, vmax, R)
    d0 = 3 * vmax * math.log(1 / R) / (2 * nbl * h)
    assert d.shape == (nz + 2 * nbl, nx + 2 * nbl)
    assert np.all(d[nbl:nbl + nz, nbl:nbl + nx] == 0.0)
    assert d[0, nbl + 5] == pytest.approx(d0)
    assert d[0, 0] == pytest.approx(2 * d0)
    assert d[nbl - 5, nbl + 3] == pytest.approx(d0 * 0.25)
    # symmetric
    assert np.allclose(d, d[::-1, :]) and np.allclose(d, d[:, ::-1])
