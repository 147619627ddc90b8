"""Pins of the oracle's two-grid interpolation, misfit and fitness."""
import math

import numpy as np
import pytest

from oracle import fd
from workloads.configs import config, true_model


def test_bilinear_reproduces_bilinear_functions():
    nz, nx, ncz, ncx = 37, 53, 4, 7
    dz = 1.0 / (nz - 1)
    # node coordinates in grid-index units
    za = np.arange(ncz) * (nz - 1) / (ncz - 1)
    xb = np.arange(ncx) * (nx - 1) / (ncx - 1)

    def f(z, x):
        return 2000.0 + 3.0 * z - 1.5 * x + 0.05 * z * x

    nodes = f(za[:, None], xb[None, :])
    vp = fd.vp_from_nodes(nodes.ravel(), ncz, ncx, nz, nx)
    i = np.arange(nz)[:, None]
    j = np.arange(nx)[None, :]
    assert np.max(np.abs(vp - f(i, j))) < 1e-9
    del dz


def test_bilinear_node_values_and_bounds():
    nz, nx, ncz, ncx = 101, 121, 5, 7     # node rows/cols fall on grid points
    rng = np.random.default_rng(1)
    nodes = rng.uniform(1400, 5000, (ncz, ncx))
    vp = fd.vp_from_nodes(nodes.ravel(), ncz, ncx, nz, nx)
    for a in range(ncz):
        for b in range(ncx):
            assert vp[a * 25, b * 20] == pytest.approx(nodes[a, b], rel=1e-14)
    assert vp.min() >= nodes.min() - 1e-9 and vp.max() <= nodes.max() + 1e-9


def test_bilinear_brute_force_single_cell():
    # hand evaluation at one interior point of a 2x2 node grid
    nodes = np.array([1000.0, 2000.0, 3000.0, 5000.0])
    vp = fd.vp_from_nodes(nodes, 2, 2, 5, 9)
    t, u = 1 / 4, 3 / 8                  # point (1, 3): z-fraction 1/4, x-fraction 3/8
    want = (1 - t) * (1 - u) * 1000 + (1 - t) * u * 2000 + t * (1 - u) * 3000 + t * u * 5000
    assert vp[1, 3] == pytest.approx(want, rel=1e-15)


def test_misfit_brute_force_and_scaling():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((3, 7, 5))
    b = rng.standard_normal((3, 7, 5))
    want = 0.5 * math.fsum(float(x) ** 2 for x in (a - b).ravel())
    assert fd.misfit(a, b) == pytest.approx(want, rel=1e-14)
    assert fd.misfit(2.5 * a, 2.5 * b) == pytest.approx(6.25 * want, rel=1e-14)
    assert fd.misfit(a, a) == 0.0


def test_fitness_zero_at_truth_and_sum_over_shots():
    g = dict(config("tiny"))
    g["src"] = [[0.0, 300.0], [0.0, 700.0]]
    prob = fd.Problem(g)
    truth = np.array([1600.0, 2000.0, 1800.0, 2400.0, 2200.0, 2600.0])
    vp = fd.vp_from_nodes(truth, 2, 3, g["nz"], g["nx"])
    d_obs = fd.forward_shots(prob, vp)
    other = truth + np.array([100.0, -50.0, 0.0, 30.0, 0.0, -80.0])
    fit, per = fd.fitness_batch(prob, np.stack([truth, other]), d_obs)
    assert fit[0] == 0.0
    assert fit[1] > 0.0
    d_other = fd.forward_shots(prob, fd.vp_from_nodes(other, 2, 3, g["nz"], g["nx"]))
    want = fd.misfit(d_other[0], d_obs[0]) + fd.misfit(d_other[1], d_obs[1])
    assert fit[1] == pytest.approx(want, rel=1e-14)
    assert per.shape == (2, 2)


def test_point_weights_on_and_off_grid():
    assert fd.point_weights((0.0, 500.0), 10.0, 10.0, 101, 101, 40) == [(40, 90, 1.0)]
    pts = fd.point_weights((15.0, 502.5), 10.0, 10.0, 101, 101, 40)
    assert sum(w for *_, w in pts) == pytest.approx(1.0)
    assert len(pts) == 4
    with pytest.raises(ValueError):
        fd.point_weights((0.0, 1001.0), 10.0, 10.0, 101, 101, 40)


def test_tiny_config_step_count():
    # the tiny workload: dt = 0.4 dt_stab at 2700 m/s, 1 s record
    prob = fd.Problem(config("tiny"))
    assert prob.dt == pytest.approx(0.4 * 0.554632 * 10.0 / 2700.0, rel=1e-6)
    assert prob.nt == 1218
    assert true_model(config("tiny")).shape == (101, 101)


def _layout(rng, L=4, nz=37, dz=10.0, nx=53, dx=12.0, rectilinear=False):
    """A layered node layout with levels strictly inside the grid and node x
    positions that need not fall on grid columns."""
    zmax, xmax = (nz - 1) * dz, (nx - 1) * dx
    node_z = np.sort(rng.uniform(0.05, 0.95, L)) * zmax
    if rectilinear:
        xs = np.sort(rng.uniform(0, xmax, 5))
        xs[0], xs[-1] = 0.0, xmax
        return node_z, [5] * L, np.tile(xs, L)
    counts = [int(c) for c in rng.integers(2, 7, L)]
    xs = []
    for c in counts:
        x = np.sort(rng.uniform(0, xmax, c))
        x[0], x[-1] = rng.uniform(0, 0.2) * xmax, rng.uniform(0.8, 1.0) * xmax
        xs.append(x)
    return node_z, counts, np.concatenate(xs)


def test_levels_reproduce_bilinear_functions_on_a_rectilinear_layout():
    rng = np.random.default_rng(21)
    nz, nx, dz, dx = 37, 53, 10.0, 12.0
    node_z, counts, node_x = _layout(rng, nz=nz, dz=dz, nx=nx, dx=dx, rectilinear=True)
    f = lambda z, x: 1800.0 + 0.7 * z - 0.3 * x + 2e-4 * z * x          # noqa: E731
    nodes = f(np.repeat(node_z, 5), node_x)
    vp = fd.vp_from_levels(nodes, node_z, counts, node_x, nz, nx, dz, dx)
    Z, X = np.meshgrid(np.arange(nz) * dz, np.arange(nx) * dx, indexing="ij")
    Zc = np.clip(Z, node_z[0], node_z[-1])                                 # constant beyond the levels
    assert np.allclose(vp, f(Zc, X), rtol=0, atol=1e-9)


def test_levels_node_values_rows_columns_and_bounds():
    rng = np.random.default_rng(22)
    nz, nx, dz, dx = 41, 61, 5.0, 8.0
    # levels on grid rows, so rows through a level can be checked directly
    node_z = np.array([6, 15, 27, 38]) * dz
    counts = [4, 3, 5, 2]
    node_x = np.concatenate([np.sort(rng.choice(np.arange(nx), c, replace=False)) * dx for c in counts])
    nodes = rng.uniform(1500, 4500, sum(counts))
    vp = fd.vp_from_levels(nodes, node_z, counts, node_x, nz, nx, dz, dx, water_rows=3, v_water=1480.0)
    starts = np.concatenate([[0], np.cumsum(counts)])
    xg = np.arange(nx) * dx
    for a in range(4):
        row = int(round(node_z[a] / dz))
        xs, vs = node_x[starts[a]:starts[a + 1]], nodes[starts[a]:starts[a + 1]]
        assert np.allclose(vp[row], np.interp(xg, xs, vs), rtol=0, atol=1e-9)     # along a level
        for b in range(counts[a]):
            assert vp[row, int(round(xs[b] / dx))] == pytest.approx(vs[b], abs=1e-9)
    # across levels at a fixed column: linear in z between the level rows
    j = 17
    lv = [vp[int(round(z / dz)), j] for z in node_z]
    zg = np.arange(nz) * dz
    below_water = zg >= 3 * dz
    assert np.allclose(vp[below_water, j], np.interp(zg[below_water], node_z, lv), rtol=0, atol=1e-9)
    assert np.all(vp[:3] == 1480.0)
    assert vp[3:].min() >= nodes.min() - 1e-9 and vp[3:].max() <= nodes.max() + 1e-9


def test_levels_brute_force_point():
    """One point worked by hand: z between levels 0 and 1, x inside a cell of each."""
    node_z = [10.0, 30.0]
    counts = [2, 3]
    node_x = [0.0, 40.0, 0.0, 20.0, 40.0]
    nodes = [1000.0, 2000.0, 3000.0, 5000.0, 4000.0]
    vp = fd.vp_from_levels(nodes, node_z, counts, node_x, 5, 5, 10.0, 10.0)
    # (z, x) = (20, 30): t = 0.5; level 0 at x = 30: 1750; level 1: 4500
    assert vp[2, 3] == pytest.approx(0.5 * 1750.0 + 0.5 * 4500.0)
    assert vp[0, 3] == pytest.approx(1750.0)                 # above the first level
    assert vp[4, 1] == pytest.approx(4000.0)                 # below the last level: level 1 at x = 10
