"""Pins of the oracle's forward modelling against closed forms, brute force and invariants."""
import math

import numpy as np
import pytest

from oracle import fd
from tests.analytic import green2d_ricker
from workloads.models import layered_faulted


def _dense_second_diff(n, w):
    D = np.zeros((n, n))
    for i in range(n):
        for k in range(-4, 5):
            if 0 <= i + k < n:
                D[i, i + k] = w[abs(k)]
    return D


def test_brute_force_dense_matrices():
    """Padded 16x16 grid, 30 steps: dense-matrix propagation vs the C loop."""
    rng = np.random.default_rng(7)
    nz = nx = 8
    nbl = 4
    Nz, Nx = nz + 2 * nbl, nx + 2 * nbl
    dz, dx = 10.0, 12.0
    vel = rng.uniform(1500, 2500, (Nz, Nx))
    damp = fd.damping_profile(nz, nx, nbl, dz, dx, 2500.0, 1e-3)
    dt = 0.4 * fd.stable_dt(2500.0, dz, dx)
    nt = 30
    wav = rng.standard_normal(nt)
    src = [(6, 7, 1.0), (9, 5, 0.5)]
    recs = [(4, 4, 1.0, 0), (10, 11, 1.0, 1), (7, 8, 0.25, 1)]
    u0 = rng.standard_normal((Nz, Nx))
    um1 = rng.standard_normal((Nz, Nx))
    tr, fin = fd.forward_run(vel, damp, dz, dx, dt, nt, wav, src, recs, 2, u0=u0, um1=um1,
                             want_final=True)

    w = [float(c) for c in fd.fd_weights(4)]
    L = (np.kron(_dense_second_diff(Nz, w), np.eye(Nx)) / dz ** 2
         + np.kron(np.eye(Nz), _dense_second_diff(Nx, w)) / dx ** 2)
    a = (0.5 * damp * dt).ravel()
    C = ((vel * dt) ** 2).ravel()
    u, up = u0.ravel().copy(), um1.ravel().copy()
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
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(tr - ref)) <= 1e-13 * scale
    assert np.max(np.abs(fin.ravel() - u)) <= 1e-13 * np.max(np.abs(u))


def _homog_problem(h, v, f0, L=1200.0, nbl_m=200.0, tmax=0.45, courant=None, dt=None):
    """Homogeneous square of side L with a centred source and an absorbing layer."""
    n = int(round(L / h)) + 1
    nbl = int(round(nbl_m / h))
    if dt is None:
        dt = courant * h / v
    nt = int(math.floor(tmax / dt + 1e-9)) + 1
    damp = fd.damping_profile(n, n, nbl, h, h, v, 1e-3)
    vel = np.full((n + 2 * nbl, n + 2 * nbl), v)
    c = (n - 1) // 2
    return n, nbl, dt, nt, damp, vel, c


def _green_errors(h, v, f0, dists, courant=None, dt=None, tmax=0.45, L=1200.0, nbl_m=200.0):
    n, nbl, dt, nt, damp, vel, c = _homog_problem(h, v, f0, L=L, nbl_m=nbl_m, courant=courant,
                                                  dt=dt, tmax=tmax)
    wav = fd.ricker(f0, dt, nt)
    recs = [(c + nbl, c + nbl + int(round(d / h)), 1.0, k) for k, d in enumerate(dists)]
    tr = fd.forward_run(vel, damp, h, h, dt, nt, wav, [(c + nbl, c + nbl, 1.0)], recs, len(dists))
    t = np.arange(nt) * dt
    errs = []
    for k, d in enumerate(dists):
        ana = green2d_ricker(d, v, f0, t)
        errs.append(np.linalg.norm(tr[:, k] - ana) / np.linalg.norm(ana))
    return errs


def test_green_function_absolute_amplitude():
    """Homogeneous medium: traces match the analytic 2-D Green's function * Ricker."""
    errs = _green_errors(5.0, 2000.0, 10.0, [100.0, 150.0, 200.0, 250.0], courant=0.4 * 0.554632)
    assert max(errs) <= 1e-2, errs


@pytest.mark.slow
def test_convergence_order_fixed_courant():
    """Refining h at a fixed Courant number: error falls at second order (time-limited)."""
    f0, v = 5.0, 2000.0
    e = [np.mean(_green_errors(h, v, f0, [200.0, 300.0], courant=0.5 * 0.554632, tmax=0.5))
         for h in (20.0, 10.0, 5.0)]
    orders = [math.log2(e[0] / e[1]), math.log2(e[1] / e[2])]
    assert min(orders) >= 1.8, (e, orders)


@pytest.mark.slow
def test_spatial_convergence_small_dt():
    """Tiny fixed dt: refining h shows the high spatial order (expected ~8, asserted >= 4)."""
    f0, v = 5.0, 2000.0
    dt = 0.05 * 0.554632 * 10.0 / v
    # large domain and thick layer: no boundary energy reaches the receiver in the window
    e = [np.mean(_green_errors(h, v, f0, [400.0], dt=dt, tmax=0.6, L=2000.0, nbl_m=400.0))
         for h in (40.0, 20.0)]
    order = math.log2(e[0] / e[1])
    assert order >= 4.0, (e, order)


def _faulted_setup():
    nz, nx, h, nbl = 61, 81, 10.0, 20
    vp = layered_faulted(nz, nx, h, h, seed=11)
    vel = fd.pad_edge(vp, nbl)
    vmax = 6000.0
    damp = fd.damping_profile(nz, nx, nbl, h, h, vmax, 1e-3)
    dt = 0.4 * fd.stable_dt(vmax, h, h)
    nt = 700
    return nz, nx, h, nbl, vel, damp, dt, nt


def test_reciprocity_heterogeneous_with_damping():
    """Swapping source and receiver gives the same trace (exact discrete reciprocity)."""
    nz, nx, h, nbl, vel, damp, dt, nt = _faulted_setup()
    wav = fd.ricker(8.0, dt, nt)
    A = (nbl + 0, nbl + 15)
    B = (nbl + 30, nbl + 60)
    tAB = fd.forward_run(vel, damp, h, h, dt, nt, wav, [(A[0], A[1], 1.0)], [(B[0], B[1], 1.0, 0)], 1)
    tBA = fd.forward_run(vel, damp, h, h, dt, nt, wav, [(B[0], B[1], 1.0)], [(A[0], A[1], 1.0, 0)], 1)
    scale = np.max(np.abs(tAB))
    assert scale > 0
    assert np.max(np.abs(tAB - tBA)) <= 1e-12 * scale


def test_mirror_symmetry():
    nz, nx, h, nbl = 41, 61, 10.0, 15
    rng = np.random.default_rng(3)
    half = rng.uniform(1500, 3000, (nz, nx // 2 + 1))
    vp = np.concatenate([half, half[:, -2::-1]], axis=1)
    assert np.allclose(vp, vp[:, ::-1])
    vel = fd.pad_edge(vp, nbl)
    damp = fd.damping_profile(nz, nx, nbl, h, h, 3000.0, 1e-3)
    dt = 0.4 * fd.stable_dt(3000.0, h, h)
    nt = 400
    wav = fd.ricker(10.0, dt, nt)
    recs = [(nbl, nbl + j, 1.0, j) for j in range(nx)]
    tr = fd.forward_run(vel, damp, h, h, dt, nt, wav, [(nbl, nbl + nx // 2, 1.0)], recs, nx)
    assert np.max(np.abs(tr - tr[:, ::-1])) <= 1e-12 * np.max(np.abs(tr))


def test_linearity_and_superposition():
    nz, nx, h, nbl, vel, damp, dt, nt = _faulted_setup()
    nt = 300
    w1 = fd.ricker(8.0, dt, nt)
    w2 = fd.ricker(5.0, dt, nt)
    S1, S2 = (nbl, nbl + 20), (nbl + 10, nbl + 50)
    recs = [(nbl, nbl + j, 1.0, k) for k, j in enumerate(range(0, nx, 5))]
    nr = len(recs)
    t1 = fd.forward_run(vel, damp, h, h, dt, nt, w1, [(S1[0], S1[1], 1.0)], recs, nr)
    t1s = fd.forward_run(vel, damp, h, h, dt, nt, 3.0 * w1, [(S1[0], S1[1], 1.0)], recs, nr)
    assert np.max(np.abs(t1s - 3.0 * t1)) <= 1e-12 * np.max(np.abs(t1s))
    # two sources driven by the same wavelet = sum of the two single-source runs
    t12 = fd.forward_run(vel, damp, h, h, dt, nt, w1, [(S1[0], S1[1], 1.0), (S2[0], S2[1], 1.0)],
                         recs, nr)
    t2 = fd.forward_run(vel, damp, h, h, dt, nt, w1, [(S2[0], S2[1], 1.0)], recs, nr)
    assert np.max(np.abs(t12 - (t1 + t2))) <= 1e-12 * np.max(np.abs(t12))
    # a different wavelet gives a different, nonzero response
    t2w = fd.forward_run(vel, damp, h, h, dt, nt, w2, [(S2[0], S2[1], 1.0)], recs, nr)
    assert np.max(np.abs(t2w)) > 0 and np.max(np.abs(t2w - t2)) > 0


def test_causality_exact_zeros():
    """The cross stencil reaches 4 points per step along one axis: earlier samples are 0."""
    nz, nx, h, nbl, vel, damp, dt, nt = _faulted_setup()
    nt = 40
    wav = fd.ricker(8.0, dt, nt)
    S = (nbl + 5, nbl + 10)
    recs = []
    for k, (di, dj) in enumerate([(0, 40), (20, 20), (9, 0), (30, 45)]):
        recs.append((S[0] + di, S[1] + dj, 1.0, k))
    tr = fd.forward_run(vel, damp, h, h, dt, nt, wav, [(S[0], S[1], 1.0)], recs, len(recs))
    for k, (di, dj) in enumerate([(0, 40), (20, 20), (9, 0), (30, 45)]):
        first = 1 + math.ceil(di / 4) + math.ceil(dj / 4)   # first step that can be nonzero
        assert np.all(tr[:first, k] == 0.0)
        assert tr[first, k] != 0.0


def test_zero_damping_inside_physical_domain():
    d = fd.damping_profile(50, 70, 20, 10.0, 10.0, 6000.0, 1e-3)
    assert np.all(d[20:70, 20:90] == 0.0)


def _box_geom(nz, nx, si, sj, offs, h=10.0):
    """Homogeneous-medium geometry without an absorbing layer: one source at
    grid point (si, sj), receivers at the given (row, column) offsets from it."""
    return {"nz": nz, "nx": nx, "dz": h, "dx": h, "nbl": 0, "vmax": 2500.0, "f0": 100.0,
            "src": [[si * h, sj * h]], "rec": [[(si + a) * h, (sj + b) * h] for a, b in offs]}


def test_grid_beyond_the_records_reach_leaves_the_traces_bit_for_bit():
    """A field that starts at the source is nonzero at step n only within
    ceil(di/4) + ceil(dj/4) <= n - 1 of it, so two grids that agree on the
    region the record reaches give identical traces whatever lies beyond: a
    source 60 points from every edge of a 121 x 121 grid, and the same source
    60 points from the bottom and right edges of a 191 x 233 grid."""
    offs = [(-6, dj) for dj in range(-12, 13, 3)]
    dt = 0.4 * fd.stable_dt(2500.0, 10.0, 10.0)
    nt = 17                                   # u^16: ceil(61/4) = 16 steps from the source, not beyond
    small = fd.Problem(_box_geom(121, 121, 60, 60, offs), dt=dt, nt=nt)
    big = fd.Problem(_box_geom(191, 233, 130, 172, offs), dt=dt, nt=nt)
    ts = fd.forward_shots(small, np.full((121, 121), 2000.0))
    tb = fd.forward_shots(big, np.full((191, 233), 2000.0))
    assert np.max(np.abs(ts)) > 0
    assert np.array_equal(ts, tb)
    # a velocity change at the source changes the traces; one just beyond
    # the field's reach does not
    vin = np.full((191, 233), 2000.0)
    vin[130, 172] = 2100.0
    vout = np.full((191, 233), 2000.0)
    vout[130, 172 - 61] = 2100.0
    assert not np.array_equal(fd.forward_shots(big, vin), tb)
    assert np.array_equal(fd.forward_shots(big, vout), tb)
