"""Pins of the oracle's misfit gradient (discrete adjoint): it must be the
exact gradient of the discrete misfit, so central finite differences of
forward_shots + misfit reproduce it to their own truncation error."""
import copy

import numpy as np
import pytest

from oracle import fd
from workloads.configs import config


def _problem():
    g = copy.deepcopy(config("tiny"))
    g.update(nz=21, nx=31, nbl=6, tmax=0.25, f0=15.0, ncz=2, ncx=3)
    g["src"] = [[0.0, 100.0], [50.0, 230.0]]
    g["rec"] = [[0.0, 10.0 * j] for j in range(0, 31, 3)]
    return g, fd.Problem(g)


def _models(op):
    z = np.arange(op.nz)[:, None] * op.dz
    x = np.arange(op.nx)[None, :] * op.dx
    vp = 1800.0 + 2.0 * z + 80.0 * np.sin(x / 90.0)
    truth = vp + 150.0 * np.exp(-((z - 110.0) ** 2 + (x - 160.0) ** 2) / 3000.0)
    return vp, truth


def _phi(op, vp, dobs):
    tr = fd.forward_shots(op, vp)
    return sum(fd.misfit(tr[s], dobs[s]) for s in range(op.nshots))


@pytest.fixture(scope="module")
def setup():
    g, op = _problem()
    vp, truth = _models(op)
    dobs = fd.forward_shots(op, truth)
    J, grad = fd.gradient(op, vp, dobs)
    return op, vp, dobs, J, grad


def test_misfit_matches_forward(setup):
    op, vp, dobs, J, grad = setup
    assert J == pytest.approx(_phi(op, vp, dobs), rel=1e-13)
    assert grad.shape == (op.nz, op.nx) and np.all(np.isfinite(grad))


@pytest.mark.parametrize("seed", [0, 1])
def test_directional_derivative_matches_central_differences(setup, seed):
    op, vp, dobs, J, grad = setup
    rng = np.random.default_rng(seed)
    z = np.arange(op.nz)[:, None]
    x = np.arange(op.nx)[None, :]
    d = np.sin(rng.uniform(0.1, 0.5) * z + rng.uniform(0, 3)) * np.cos(rng.uniform(0.1, 0.4) * x + rng.uniform(0, 3))
    eps = 0.05                                                   # m/s along d (|d| <= 1)
    fd_val = (_phi(op, vp + eps * d, dobs) - _phi(op, vp - eps * d, dobs)) / (2 * eps)
    assert np.sum(grad * d) == pytest.approx(fd_val, rel=1e-6)


@pytest.mark.parametrize("ij", [(10, 15), (0, 0), (0, 12), (20, 30), (5, 21)])
def test_pointwise_derivative_matches_central_differences(setup, ij):
    """Interior point, corners (which the absorbing layer copies), receiver row."""
    op, vp, dobs, J, grad = setup
    e = np.zeros_like(vp)
    e[ij] = 1.0
    eps = 0.05
    fd_val = (_phi(op, vp + eps * e, dobs) - _phi(op, vp - eps * e, dobs)) / (2 * eps)
    assert grad[ij] == pytest.approx(fd_val, rel=1e-5, abs=1e-9 * np.abs(grad).max())


def test_zero_residual_gives_zero_gradient(setup):
    op, vp, dobs, J, grad = setup
    d0 = fd.forward_shots(op, vp)
    J0, g0 = fd.gradient(op, vp, d0)
    assert J0 == 0.0 and np.all(g0 == 0.0)


def test_unpad_adjoint_is_the_transpose_of_pad_edge():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((7, 9))
    b = rng.standard_normal((7 + 6, 9 + 6))
    assert np.sum(fd.pad_edge(a, 3) * b) == pytest.approx(np.sum(a * fd.unpad_adjoint(b, 3)), rel=1e-13)
