"""Pin of the oracle's absorbing layer as a physical absorber.

The same source and receivers are modelled in a 1 km grid with the damping
layer and in a 6 km grid whose edges are too far for any echo to return
within the 1.5 s record; the difference of the two records is what the small
grid's layer reflects. With the 40-point quadratic profile it stays under 3 %
of the record (1.9 % measured), grows as the layer thins, and exceeds the
record itself without a layer. Three plausible mistakes in the profile
(damping along x only, a peak damping ten times too weak or too strong) reflect
more than the bar.
"""
import copy

import numpy as np
import pytest

from oracle import fd
from workloads.configs import config

BAR = 0.03


def _geom(n, off, nbl):
    g = copy.deepcopy(config("tiny"))
    g.update(nz=n, nx=n, dz=10.0, dx=10.0, nbl=nbl, f0=15.0, tmax=1.5)
    g["src"] = [[off + 500.0, off + 500.0]]
    g["rec"] = [[off + 500.0, off + 10.0 * j] for j in (10, 20, 30, 70, 80, 90)]
    return g


@pytest.fixture(scope="module")
def far():
    """Records of the 6 km grid (source 3 km from every edge: echoes need 3 s)."""
    small = fd.Problem(_geom(101, 0.0, 40))
    big = fd.Problem(_geom(601, 2500.0, 40), dt=small.dt, nt=small.nt)
    return small.dt, small.nt, fd.forward_shots(big, np.full((601, 601), 2000.0))[0]


def _reflected(far, nbl):
    dt, nt, ref = far
    p = fd.Problem(_geom(101, 0.0, nbl), dt=dt, nt=nt)
    tr = fd.forward_shots(p, np.full((101, 101), 2000.0))[0]
    return float(np.linalg.norm(tr - ref) / np.linalg.norm(ref))


def test_layer_reflects_little_and_less_as_it_thickens(far):
    e40, e20, e0 = _reflected(far, 40), _reflected(far, 20), _reflected(far, 0)
    assert e40 < BAR, e40
    assert e40 < e20 < e0 and e0 > 1.0, (e40, e20, e0)


def _x_only(real):
    def prof(nz, nx, nbl, dz, dx, vmax, R=1e-3):
        d = real(nz, nx, nbl, dz, dx, vmax, R)
        return d - d[:, nbl + nx // 2][:, None]          # the x part alone: the z part is 0 at mid-x
    return prof


@pytest.mark.parametrize("name", ["x only", "peak / 10", "peak x 10"])
def test_planted_profile_mistake_is_caught(far, monkeypatch, name):
    real = fd.damping_profile
    mutant = {"x only": _x_only(real),
              "peak / 10": lambda *a, **k: real(*a, **k) / 10.0,
              "peak x 10": lambda *a, **k: real(*a, **k) * 10.0}[name]
    monkeypatch.setattr(fd, "damping_profile", mutant)
    assert _reflected(far, 40) > BAR
