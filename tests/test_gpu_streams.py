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


def test_calls_from_two_host_threads_equal_sequential_ones(gfd):  # noqa: F811  (the imported fixture)
    """The library's caches (launch plans, tunings, the second stream) are
    shared by host threads under a lock and its error text is per thread:
    two threads, each with its own stream and workspaces, evaluating
    fitness batches and gradients concurrently get the sequential results
    bit for bit."""
    import threading
    g = _small_geom()
    op, gp = _pair(gfd, g)
    rng = np.random.default_rng(32)
    dobs = torch.tensor(rng.standard_normal((3, gp.nt, gp.nrec)).astype(np.float32) * 1e-3, device="cuda")
    sets = [[rng.uniform(1400, 2700, (4 + t, 12)) for _ in range(3)] for t in range(2)]
    w = _wide()
    opw = ofd.Problem(w)
    gw = gfd.Problem(w, dt=opw.dt, nt=opw.nt)
    vp, truth = _models(opw.nz, opw.nx, opw.dz, opw.dx)
    obs = torch.tensor(ofd.forward_shots(opw, truth).astype(np.float32), device="cuda")
    models = [torch.tensor(vp, dtype=torch.float32, device="cuda"),
              torch.tensor(0.5 * (vp + truth), dtype=torch.float32, device="cuda")]
    fbs = [gfd.FitnessBatch([gp], [dobs], [0] * (4 + t)) for t in range(2)]
    want = [[fbs[t](X).clone() for X in sets[t]] for t in range(2)]
    want_g = [tuple(x.clone() for x in gfd.gradient(gw, models[t], obs)) for t in range(2)]
    torch.cuda.synchronize()
    got = [[None] * 3 for _ in range(2)]
    got_g = [None, None]
    errors = []

    def work(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for k in range(3):
                    got[t][k] = fbs[t](sets[t][k]).clone()
                got_g[t] = tuple(x.clone() for x in gfd.gradient(gw, models[t], obs))
            s.synchronize()
        except Exception as e:                      # reported by the main thread
            errors.append(repr(e))

    th = [threading.Thread(target=work, args=(t,), daemon=True) for t in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=120)
    torch.cuda.synchronize()
    assert not errors and not any(x.is_alive() for x in th), errors
    for t in range(2):
        for k in range(3):
            assert torch.equal(got[t][k], want[t][k]), (t, k)
        assert torch.equal(got_g[t][0], want_g[t][0]) and torch.equal(got_g[t][1], want_g[t][1]), t
