"""The oracle's pins catch plausible mistakes (mistakes are planted in a copy of the oracle, on the CPU).

Each case compiles a copy of oracle_fd.c with one plausible error, or patches
one oracle helper, and checks that a pin from the oracle test suite fails on
it while passing on the real oracle.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import build as obuild
from oracle import fd
from tests.analytic import green2d_ricker

SRC = open(obuild.SRC).read()

MUTATIONS = {
    "damping sign": ("double a = 0.5 * damp[IDX(I, J)] * dt;", "double a = -0.5 * damp[IDX(I, J)] * dt;"),
    "dz and dx swapped": ("const double idz2 = 1.0 / (dz * dz), idx2 = 1.0 / (dx * dx);",
                          "const double idz2 = 1.0 / (dx * dx), idx2 = 1.0 / (dz * dz);"),
    "source without 1/(dz dx)": ("unext[q] += C * sw[p] * wavelet[n] / (dz * dx) / (1.0 + a);",
                                 "unext[q] += C * sw[p] * wavelet[n] / (1.0 + a);"),
    "sampling after the update": ("        if (n == nt - 1) break;\n",
                                  "        if (n == nt - 1) break;\n        if (traces) for (int r = 0; r < nrec; ++r) traces[(size_t)n * nrec + r] = 0.0;\n"
                                  "        if (traces) for (int p = 0; p < nrp; ++p) traces[(size_t)n * nrec + rid[p]] += rw[p] * u[IDX(rI[p], rJ[p]) + 1];\n"),
    "neighbour index off by one": ("double rt = (J + k < Nx) ? u[IDX(I, J + k)] : 0.0;",
                                   "double rt = (J + k + 1 < Nx) ? u[IDX(I, J + k + 1)] : 0.0;"),
}


def _mutant_lib(tmp_path, name):
    old, new = MUTATIONS[name]
    assert old in SRC, name
    src = tmp_path / "m.c"
    src.write_text(SRC.replace(old, new, 1))
    so = tmp_path / "m.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", str(so), str(src)])
    lib = ctypes.CDLL(str(so))
    lib.oracle_forward_run.restype = ctypes.c_int
    lib.oracle_forward_run.argtypes = fd._load().oracle_forward_run.argtypes
    return lib


def _brute_force_error(vel_dz=10.0, vel_dx=12.0):
    """Max relative deviation of the C loop from the dense-matrix propagation (test_oracle_forward)."""
    from tests.test_oracle_forward import _dense_second_diff
    rng = np.random.default_rng(7)
    nz = nx = 8
    nbl = 4
    Nz, Nx = nz + 2 * nbl, nx + 2 * nbl
    dz, dx = vel_dz, vel_dx
    vel = rng.uniform(1500, 2500, (Nz, Nx))
    damp = fd.damping_profile(nz, nx, nbl, dz, dx, 2500.0, 1e-3)
    dt = 0.4 * fd.stable_dt(2500.0, dz, dx)
    nt = 30
    wav = rng.standard_normal(nt)
    src = [(6, 7, 1.0)]
    recs = [(4, 4, 1.0, 0), (10, 11, 1.0, 1)]
    u0 = rng.standard_normal((Nz, Nx))
    tr = fd.forward_run(vel, damp, dz, dx, dt, nt, wav, src, recs, 2, u0=u0, um1=u0)
    w = [float(c) for c in fd.fd_weights(4)]
    L = (np.kron(_dense_second_diff(Nz, w), np.eye(Nx)) / dz ** 2
         + np.kron(np.eye(Nz), _dense_second_diff(Nx, w)) / dx ** 2)
    a = (0.5 * damp * dt).ravel()
    C = ((vel * dt) ** 2).ravel()
    u, up = u0.ravel().copy(), u0.ravel().copy()
    ref = np.zeros((nt, 2))
    for n in range(nt):
        for (I, J, ww, r) in recs:
            ref[n, r] += ww * u[I * Nx + J]
        if n == nt - 1:
            break
        f = np.zeros(Nz * Nx)
        for (I, J, ww) in src:
            f[I * Nx + J] += ww * wav[n] / (dz * dx)
        un = (2 * u - (1 - a) * up + C * (L @ u + f)) / (1 + a)
        up, u = u, un
    return float(np.max(np.abs(tr - ref)) / np.max(np.abs(ref)))


def _green_error():
    h, v, f0 = 5.0, 2000.0, 10.0
    n, nbl = 241, 40
    dt = 0.4 * 0.554632 * h / v
    nt = int(math.floor(0.45 / dt + 1e-9)) + 1
    damp = fd.damping_profile(n, n, nbl, h, h, v, 1e-3)
    vel = np.full((n + 2 * nbl, n + 2 * nbl), v)
    c = (n - 1) // 2
    wav = fd.ricker(f0, dt, nt)
    tr = fd.forward_run(vel, damp, h, h, dt, nt, wav, [(c + nbl, c + nbl, 1.0)],
                        [(c + nbl, c + nbl + 30, 1.0, 0)], 1)
    ana = green2d_ricker(150.0, v, f0, np.arange(nt) * dt)
    return float(np.linalg.norm(tr[:, 0] - ana) / np.linalg.norm(ana))


def test_real_oracle_passes_the_pins():
    assert _brute_force_error() <= 1e-13
    assert _green_error() <= 1e-2


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, monkeypatch, name):
    lib = _mutant_lib(tmp_path, name)
    monkeypatch.setattr(fd, "_lib", lib)
    caught = _brute_force_error() > 1e-6 or _green_error() > 1e-2
    assert caught, name


def test_planted_ricker_delay_is_caught(monkeypatch):
    real = fd.ricker
    monkeypatch.setattr(fd, "ricker", lambda f0, dt, nt, t0=None: real(f0, dt, nt, t0=0.5 / f0))
    assert _green_error() > 1e-2


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_planted_weight_sign_error_is_caught(monkeypatch, k):
    real = fd.fd_weights(4)
    bad = list(real)
    bad[k] = -bad[k]
    monkeypatch.setattr(fd, "fd_weights", lambda M=4: bad)
    err = _green_error()
    assert not (err <= 1e-2), err          # large or non-finite


LEVEL_MUTATIONS = {
    "z weights swapped": ("out[i, j] = (1.0 - t) * along(a, x) + t * along(a + 1, x)",
                          "out[i, j] = t * along(a, x) + (1.0 - t) * along(a + 1, x)"),
    "x weights swapped": ("return (1.0 - u) * vs[b] + u * vs[b + 1]", "return u * vs[b] + (1.0 - u) * vs[b + 1]"),
    "z measured from the wrong level": ("t = (z - node_z[a]) / (node_z[a + 1] - node_z[a])",
                                        "t = (z - node_z[a + 1]) / (node_z[a + 1] - node_z[a])"),
    "last level not clamped": ("a, t = L - 2, 1.0", "a, t = L - 2, 0.0"),
    "water rows ignored": ("        if i < water_rows:\n", "        if i < 0:\n"),
}


@pytest.mark.parametrize("name", sorted(LEVEL_MUTATIONS))
def test_planted_level_interpolation_mistake_is_caught(monkeypatch, name):
    import inspect
    import textwrap

    from tests import test_oracle_model as pins
    old, new = LEVEL_MUTATIONS[name]
    src = textwrap.dedent(inspect.getsource(fd.vp_from_levels))
    assert old in src, name
    ns = dict(fd.__dict__)
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    monkeypatch.setattr(fd, "vp_from_levels", ns["vp_from_levels"])
    caught = 0
    for pin in (pins.test_levels_reproduce_bilinear_functions_on_a_rectilinear_layout,
                pins.test_levels_node_values_rows_columns_and_bounds, pins.test_levels_brute_force_point):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught > 0, name


GRADIENT_MUTATIONS = {
    "residual injected with the wrong sign": ("p0[q] += C * rw[p] * res[(size_t)k * nrec + rid[p]] / (1.0 + a);",
                                              "p0[q] -= C * rw[p] * res[(size_t)k * nrec + rid[p]] / (1.0 + a);"),
    "residual of the wrong time sample": ("p0[q] += C * rw[p] * res[(size_t)k * nrec + rid[p]] / (1.0 + a);",
                                          "p0[q] += C * rw[p] * res[(size_t)(k - 1) * nrec + rid[p]] / (1.0 + a);"),
    "adjoint without damping": ("p0[IDX(I, J)] = (2.0 * p1[IDX(I, J)] - (1.0 - a) * p2[IDX(I, J)]",
                                "p0[IDX(I, J)] = (2.0 * p1[IDX(I, J)] - p2[IDX(I, J)]"),
    "imaging term one level late": ("double second = (1.0 + a) * uk[q] - 2.0 * uk1[q] + (1.0 - a) * (uk2 ? uk2[q] : 0.0);",
                                    "double second = (1.0 + a) * uk1[q] - 2.0 * (uk2 ? uk2[q] : 0.0);"),
}


@pytest.mark.parametrize("name", sorted(GRADIENT_MUTATIONS))
def test_planted_adjoint_mistake_is_caught(tmp_path, monkeypatch, name):
    from tests import test_oracle_gradient as pins
    old, new = GRADIENT_MUTATIONS[name]
    assert old in SRC, name
    src = tmp_path / "m.c"
    src.write_text(SRC.replace(old, new, 1))
    so = tmp_path / "m.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", str(so), str(src)])
    lib = ctypes.CDLL(str(so))
    real = fd._load()
    for fn in ("oracle_forward_run", "oracle_gradient_run"):
        getattr(lib, fn).restype = ctypes.c_int
        getattr(lib, fn).argtypes = getattr(real, fn).argtypes
    monkeypatch.setattr(fd, "_lib", lib)
    g, op = pins._problem()
    vp, truth = pins._models(op)
    dobs = fd.forward_shots(op, truth)
    J, grad = fd.gradient(op, vp, dobs)
    z = np.arange(op.nz)[:, None]
    x = np.arange(op.nx)[None, :]
    d = np.sin(0.3 * z + 1.0) * np.cos(0.2 * x + 0.5)
    eps = 0.05
    fd_val = (pins._phi(op, vp + eps * d, dobs) - pins._phi(op, vp - eps * d, dobs)) / (2 * eps)
    assert abs(np.sum(grad * d) - fd_val) > 1e-4 * abs(fd_val), name
