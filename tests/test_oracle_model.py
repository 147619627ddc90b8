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
