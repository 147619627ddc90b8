"""Pins of the oracle's trace-normalised misfit and of its gradient.

Each trace (one receiver of one shot over time) of the modelled and of the
observed data is divided by its own l2 norm, or by the floor w = 1e-4 times
the largest trace norm of the same shot and side where that is larger, before
the l2 misfit; a zero trace stays zero. Pinned by hand-worked examples (above and
below the floor), the cosine identity
1/2 |a/|a| - b/|b||^2 = 1 - cos(a, b), the special cases (parallel,
antiparallel, orthogonal, zero traces), invariance under a positive scale of
any single trace, finite differences of the misfit with respect to the traces
(the adjoint data), and central finite differences of the whole chain
model -> traces -> misfit (the gradient). Planted mistakes fail these pins.
"""
import copy

import numpy as np
import pytest

from oracle import fd
from workloads.configs import config


def test_worked_example():
    # one receiver, two samples: d = (3, 4), o = (1, 0): d/|d| = (0.6, 0.8),
    # 1/2 ((0.6 - 1)^2 + 0.8^2) = 1/2 (0.16 + 0.64) = 0.4
    d = np.array([[3.0], [4.0]])
    o = np.array([[1.0], [0.0]])
    assert fd.misfit_normalised(d, o) == pytest.approx(0.4, abs=1e-15)
    # two receivers: the second one (d = (0, 2), o = (5, 5)) adds 1 - 1/sqrt(2)
    d2 = np.array([[3.0, 0.0], [4.0, 2.0]])
    o2 = np.array([[1.0, 5.0], [0.0, 5.0]])
    assert fd.misfit_normalised(d2, o2) == pytest.approx(0.4 + 1.0 - 2 ** -0.5, abs=1e-15)


def test_worked_example_below_the_floor():
    # observed norms 10 and 5e-4 -> wo = 1e-3: o_hat = (1, 0) and (0, 5e-4)/1e-3 = (0, 0.5);
    # modelled norms 5 and 2e-4 -> wd = 5e-4: (3, 4) -> (0.6, 0.8), (0, 2e-4)/5e-4 = (0, 0.4);
    # 1/2 ((0.6 - 1)^2 + 0.8^2) + 1/2 (0.4 - 0.5)^2 = 0.4 + 0.005
    o = np.array([[10.0, 0.0], [0.0, 5e-4]])
    d = np.array([[3.0, 0.0], [4.0, 2e-4]])
    assert fd.trace_floor(o) == pytest.approx(1e-3, rel=1e-15)
    assert fd.trace_floor(d) == pytest.approx(5e-4, rel=1e-15)
    assert fd.misfit_normalised(d, o) == pytest.approx(0.405, abs=1e-14)


def test_cosine_identity_on_random_traces():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((50, 7))
    b = rng.standard_normal((50, 7))
    cos = [np.dot(a[:, r], b[:, r]) / (np.linalg.norm(a[:, r]) * np.linalg.norm(b[:, r])) for r in range(7)]
    assert fd.misfit_normalised(a, b) == pytest.approx(sum(1.0 - c for c in cos), rel=1e-13)


def test_special_cases():
    rng = np.random.default_rng(5)
    o = rng.standard_normal((40, 3))
    assert fd.misfit_normalised(2.5 * o, o) == pytest.approx(0.0, abs=1e-14)       # parallel
    assert fd.misfit_normalised(-o, o) == pytest.approx(2.0 * 3, rel=1e-14)        # antiparallel
    t = np.arange(40)
    a = np.stack([np.sin(2 * np.pi * t / 40), np.cos(2 * np.pi * t / 40)], axis=1)
    b = np.stack([np.cos(2 * np.pi * t / 40), np.sin(2 * np.pi * t / 40)], axis=1)
    assert fd.misfit_normalised(a, b) == pytest.approx(2.0, abs=1e-13)             # orthogonal: 1 each
    z = np.zeros((40, 3))
    assert fd.misfit_normalised(z, o) == pytest.approx(0.5 * 3, rel=1e-15)         # zero modelled trace
    assert fd.misfit_normalised(o, z) == pytest.approx(0.5 * 3, rel=1e-15)         # zero observed trace
    assert fd.misfit_normalised(z, z) == 0.0
    bad = o.copy()
    bad[3, 1] = np.nan
    assert fd.misfit_normalised(bad, o) == np.inf


def test_invariant_under_a_scale_of_any_trace():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((3, 60, 5))                                            # [shot][nt][nrec]
    b = rng.standard_normal((3, 60, 5))
    m = fd.misfit_normalised(a, b)
    sa = rng.uniform(0.1, 10.0, size=(3, 1, 5))                                   # all stay above the floor
    sb = rng.uniform(0.1, 10.0, size=(3, 1, 5))
    assert fd.misfit_normalised(a * sa, b * sb) == pytest.approx(m, rel=1e-12)
    # and under a scale of all traces of one side, far beyond the floor's ratio
    assert fd.misfit_normalised(a * 1e-12, b * 1e9) == pytest.approx(m, rel=1e-12)
    # a scale along time (the other axis) does change it
    st = rng.uniform(0.5, 2.0, size=(1, 60, 1))
    assert abs(fd.misfit_normalised(a * st, b) - m) > 1e-3 * m


def test_adjoint_data_is_the_derivative_of_the_misfit():
    rng = np.random.default_rng(11)
    d = rng.standard_normal((30, 4))
    o = rng.standard_normal((30, 4))
    o[:, 2] = 0.0                                                                  # a zero observed trace
    d[:, 1] *= 1e-6                                                                # a modelled trace below the floor
    d[:, 3] *= 3.0                                                                 # the largest modelled trace
    assert np.linalg.norm(d[:, 1]) < fd.trace_floor(d)
    assert int(np.argmax(np.linalg.norm(d, axis=0))) == 3
    g = d - fd.normalised_adjoint_data(d, o)
    h = 1e-6
    for (n, r) in [(0, 0), (7, 1), (29, 3), (5, 3), (12, 2), (3, 1)]:
        e = np.zeros_like(d)
        e[n, r] = h
        num = (fd.misfit_normalised(d + e, o) - fd.misfit_normalised(d - e, o)) / (2 * h)
        assert g[n, r] == pytest.approx(num, rel=1e-6, abs=1e-10)


def _problem():
    g = copy.deepcopy(config("tiny"))
    g.update(nz=21, nx=31, nbl=6, tmax=0.25, f0=15.0, ncz=2, ncx=3, misfit="trace_normalised")
    g["src"] = [[0.0, 100.0], [50.0, 230.0]]
    g["rec"] = [[0.0, 10.0 * j] for j in range(0, 31, 3)]
    return fd.Problem(g)


def _models(op):
    z = np.arange(op.nz)[:, None] * op.dz
    x = np.arange(op.nx)[None, :] * op.dx
    vp = 1800.0 + 2.0 * z + 80.0 * np.sin(x / 90.0)
    truth = vp + 150.0 * np.exp(-((z - 110.0) ** 2 + (x - 160.0) ** 2) / 3000.0)
    return vp, truth


def _phi(op, vp, dobs):
    tr = fd.forward_shots(op, vp)
    return sum(fd.misfit_normalised(tr[s], dobs[s]) for s in range(op.nshots))


@pytest.fixture(scope="module")
def setup():
    op = _problem()
    vp, truth = _models(op)
    # observed data of unknown amplitude: the true traces times a factor per shot
    dobs = fd.forward_shots(op, truth) * np.array([3.7, 0.2])[:, None, None]
    J, grad = fd.gradient(op, vp, dobs)
    return op, vp, truth, dobs, J, grad


def test_gradient_misfit_matches_forward(setup):
    op, vp, truth, dobs, J, grad = setup
    assert J == pytest.approx(_phi(op, vp, dobs), rel=1e-13)
    assert J > 0 and np.all(np.isfinite(grad))


def test_true_model_fits_scaled_data_exactly(setup):
    op, vp, truth, dobs, J, grad = setup
    assert _phi(op, truth, dobs) == pytest.approx(0.0, abs=1e-12)
    f, _ = fd.fitness_batch(op, np.full((1, op.D), 2000.0), dobs)
    assert f[0] == pytest.approx(_phi(op, np.full((op.nz, op.nx), 2000.0), dobs), rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_directional_derivative_matches_central_differences(setup, seed):
    op, vp, truth, dobs, J, grad = setup
    rng = np.random.default_rng(seed)
    z = np.arange(op.nz)[:, None]
    x = np.arange(op.nx)[None, :]
    d = np.sin(rng.uniform(0.1, 0.5) * z + rng.uniform(0, 3)) * np.cos(rng.uniform(0.1, 0.4) * x + rng.uniform(0, 3))
    eps = 0.05
    fd_val = (_phi(op, vp + eps * d, dobs) - _phi(op, vp - eps * d, dobs)) / (2 * eps)
    assert np.sum(grad * d) == pytest.approx(fd_val, rel=1e-6)


@pytest.mark.parametrize("ij", [(10, 15), (0, 0), (0, 12)])
def test_pointwise_derivative_matches_central_differences(setup, ij):
    op, vp, truth, dobs, J, grad = setup
    e = np.zeros_like(vp)
    e[ij] = 1.0
    eps = 0.05
    fd_val = (_phi(op, vp + eps * e, dobs) - _phi(op, vp - eps * e, dobs)) / (2 * eps)
    assert grad[ij] == pytest.approx(fd_val, rel=1e-5, abs=1e-9 * np.abs(grad).max())


# ---- planted mistakes --------------------------------------------------------

def _normalise_over_receivers(d, w):
    d = np.asarray(d, dtype=np.float64)
    nrm = np.maximum(np.sqrt(np.sum(d * d, axis=-1, keepdims=True)), w)
    return np.divide(d, nrm, out=np.zeros_like(d), where=nrm > 0)


def test_planted_normalisation_axis_mistake_is_caught(monkeypatch):
    monkeypatch.setattr(fd, "normalise_traces", _normalise_over_receivers)
    with pytest.raises(AssertionError):
        test_invariant_under_a_scale_of_any_trace()


def test_planted_missing_projection_is_caught(monkeypatch):
    def bad(d, o):
        oh = fd.normalise_traces(o, fd.trace_floor(o))
        n = np.maximum(np.sqrt(np.sum(d * d, axis=0)), fd.trace_floor(d))
        return d - (d / n - oh) / n                                               # (I - e e^T) dropped
    monkeypatch.setattr(fd, "normalised_adjoint_data", bad)
    with pytest.raises(AssertionError):
        test_adjoint_data_is_the_derivative_of_the_misfit()


def test_planted_missing_floor_derivative_is_caught(monkeypatch):
    real = fd.normalised_adjoint_data

    def bad(d, o):
        out = real(d, o)
        # undo the floor term: recompute trace k's derivative without it
        w = fd.trace_floor(d)
        oh = fd.normalise_traces(o, fd.trace_floor(o))
        k = int(np.argmax(np.linalg.norm(d, axis=0)))
        x, y = d[:, k], oh[:, k]
        n = np.linalg.norm(x)
        e = x / n
        out[:, k] = x - ((e - y) - e * np.dot(e, e - y)) / n
        return out
    monkeypatch.setattr(fd, "normalised_adjoint_data", bad)
    with pytest.raises(AssertionError):
        test_adjoint_data_is_the_derivative_of_the_misfit()


def test_planted_missing_floor_is_caught(monkeypatch):
    monkeypatch.setattr(fd, "TRACE_FLOOR", 0.0)
    with pytest.raises(AssertionError):
        test_worked_example_below_the_floor()


def test_planted_shared_floor_is_caught(monkeypatch):
    """A floor taken from the observed side for both sides breaks the scale invariance."""
    def bad(a, b):
        a = np.asarray(a, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        if a.ndim == 3:
            return float(sum(bad(a[s], b[s]) for s in range(a.shape[0])))
        w = fd.trace_floor(b)
        return fd.misfit(fd.normalise_traces(a, w), fd.normalise_traces(b, w))
    monkeypatch.setattr(fd, "misfit_normalised", bad)
    with pytest.raises(AssertionError):
        test_invariant_under_a_scale_of_any_trace()
