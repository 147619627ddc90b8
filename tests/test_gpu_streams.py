"""Overlapping calls on two streams (run on an MI355X)."""
import numpy as np
import pytest
import torch

from oracle import fd as ofd
from tests.test_gpu_fd import _pair, _small_geom, gfd  # noqa: F401  (fixture)
from tests.test_gpu_gradient import _models, _wide

pytestmark = pytest.mark.gpu


def test_overlapping_calls_on_two_streams_equal_sequential_ones(gfd):  # noqa: F811  (the imported fixture)
    """Problems are shared between streams; calls that overlap on different
    streams with their own workspaces give what the same calls give one after
    another, bit for bit: two fitness batches of one problem, and two
    gradients (whose segment recomputation shares the library's second
    stream), each pair enqueued on two streams of default priority."""
    g = _small_geom()
    op, gp = _pair(gfd, g)
    rng = np.random.default_rng(31)
    dobs = torch.tensor(rng.standard_normal((3, gp.nt, gp.nrec)).astype(np.float32) * 1e-3, device="cuda")
    XA, XB = rng.uniform(1400, 2700, (6, 12)), rng.uniform(1400, 2700, (9, 12))
    fa = gfd.FitnessBatch([gp], [dobs], [0] * 6)
    fbb = gfd.FitnessBatch([gp], [dobs], [0] * 9)
    ra, rb = fa(XA).clone(), fbb(XB).clone()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(s1):
            oa = fa(XA)
        with torch.cuda.stream(s2):
            ob = fbb(XB)
        torch.cuda.synchronize()
        assert torch.equal(oa, ra) and torch.equal(ob, rb)

    w = _wide()
    opw = ofd.Problem(w)
    gw = gfd.Problem(w, dt=opw.dt, nt=opw.nt)
    vp, truth = _models(opw.nz, opw.nx, opw.dz, opw.dx)
    obs = torch.tensor(ofd.forward_shots(opw, truth).astype(np.float32), device="cuda")
    v1 = torch.tensor(vp, dtype=torch.float32, device="cuda")
    v2 = torch.tensor(0.5 * (vp + truth), dtype=torch.float32, device="cuda")
    m1, g1 = (t.clone() for t in gfd.gradient(gw, v1, obs))
    m2, g2 = (t.clone() for t in gfd.gradient(gw, v2, obs))
    assert not torch.equal(g1, g2)
    torch.cuda.synchronize()
    for _ in range(2):
        with torch.cuda.stream(s1):
            a = gfd.gradient(gw, v1, obs)
        with torch.cuda.stream(s2):
            b = gfd.gradient(gw, v2, obs)
        torch.cuda.synchronize()
        assert torch.equal(a[0], m1) and torch.equal(a[1], g1)
        assert torch.equal(b[0], m2) and torch.equal(b[1], g2)
